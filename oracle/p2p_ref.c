/*
 * Plain FP64 pair sums of the MFS representation -- test infrastructure only.
 *
 * This file belongs to the CPU oracle.  It is compiled on its own (gcc) and is
 * loaded only by the tests, by the smoke check and by the CPU-baseline leg of
 * the benchmark; the GPU library never links or calls it.
 *
 * Each routine is the literal definition: a double loop over every target and
 * every source, one fundamental solution per pair, summed in FP64.  The only
 * concession to speed is an OpenMP split over targets (each target's sum is
 * still taken over sources in index order).
 *
 *   Laplace (Section 2.1):   G(x, y) = 1 / (4 pi |x - y|)
 *   Stokes  (Section 2.2, the Stokeslet):
 *       G(x, y) = (I + (x - y)(x - y)^T / |x - y|^2) / (8 pi mu |x - y|)
 *   Representation (eqs. for u as a sum over bodies and proxies):
 *       u(x_i) = sum_j G(x_i, y_j) s_j
 *
 * With skip_same_body != 0 a pair whose target and source carry the same body
 * id is left out (the off-diagonal blocks S^(kk'), k' != k, of the MFS matrix).
 * Points are [n][3] row-major, strengths [n] (Laplace) or [n][3] (Stokes).
 */
#include <math.h>
#include <stdint.h>

static const double PI = 3.14159265358979323846;

void oracle_p2p_laplace(int64_t n_trg, const double *x, const int32_t *trg_body,
                        int64_t n_src, const double *y, const int32_t *src_body,
                        const double *q, int skip_same_body, double *u)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_trg; ++i) {
        double sum = 0.0;
        for (int64_t j = 0; j < n_src; ++j) {
            if (skip_same_body && trg_body[i] == src_body[j])
                continue;
            double d0 = x[3 * i + 0] - y[3 * j + 0];
            double d1 = x[3 * i + 1] - y[3 * j + 1];
            double d2 = x[3 * i + 2] - y[3 * j + 2];
            double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            double G = 1.0 / (4.0 * PI * r);
            sum += G * q[j];
        }
        u[i] = sum;
    }
}

void oracle_p2p_stokes(int64_t n_trg, const double *x, const int32_t *trg_body,
                       int64_t n_src, const double *y, const int32_t *src_body,
                       const double *f, double mu, int skip_same_body, double *u)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_trg; ++i) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int64_t j = 0; j < n_src; ++j) {
            if (skip_same_body && trg_body[i] == src_body[j])
                continue;
            double d[3] = {x[3 * i + 0] - y[3 * j + 0],
                           x[3 * i + 1] - y[3 * j + 1],
                           x[3 * i + 2] - y[3 * j + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            double pref = 1.0 / (8.0 * PI * mu * r);
            double G[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    G[a][b] = pref * ((a == b ? 1.0 : 0.0) + d[a] * d[b] / r2);
            const double *fj = f + 3 * j;
            s0 += G[0][0] * fj[0] + G[0][1] * fj[1] + G[0][2] * fj[2];
            s1 += G[1][0] * fj[0] + G[1][1] * fj[1] + G[1][2] * fj[2];
            s2 += G[2][0] * fj[0] + G[2][1] * fj[1] + G[2][2] * fj[2];
        }
        u[3 * i + 0] = s0;
        u[3 * i + 1] = s1;
        u[3 * i + 2] = s2;
    }
}

/*
 * Gradients of the pairing  Phi = sum_i sum_j w_i . G(x_i - y_j) s_j  with
 * respect to every target position x_i (gx) and every source position y_j
 * (gy), same pair set as above.  With d = x - y, r = |d|:
 *   Laplace: dPhi_ij/dd = -w_i s_j d / (4 pi r^3)
 *   Stokes:  dPhi_ij/dd = [ -(w.s) d + (w.d) s + (s.d) w - 3 (w.d)(s.d) d / r^2 ] / (8 pi mu r^3)
 * and dPhi/dx_i = sum_j dPhi_ij/dd,  dPhi/dy_j = -sum_i dPhi_ij/dd.
 * Written as two plain loops (one per output) so that neither needs atomics.
 */
static void stokes_pair_grad(const double *d, const double *w, const double *s, double mu, double *g)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    double ws = w[0] * s[0] + w[1] * s[1] + w[2] * s[2];
    double wd = w[0] * d[0] + w[1] * d[1] + w[2] * d[2];
    double sd = s[0] * d[0] + s[1] * d[1] + s[2] * d[2];
    double c = 1.0 / (8.0 * PI * mu * r * r2);
    for (int a = 0; a < 3; ++a)
        g[a] = c * (-ws * d[a] + wd * s[a] + sd * w[a] - 3.0 * wd * sd * d[a] / r2);
}

static void laplace_pair_grad(const double *d, double w, double s, double *g)
{
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double r = sqrt(r2);
    double c = -w * s / (4.0 * PI * r * r2);
    for (int a = 0; a < 3; ++a)
        g[a] = c * d[a];
}

void oracle_p2p_grad(int kind, int64_t n_trg, const double *x, const int32_t *trg_body,
                     const double *w, int64_t n_src, const double *y, const int32_t *src_body,
                     const double *s, double mu, int skip_same_body, double *gx, double *gy)
{
    const int dim = kind ? 3 : 1;
    if (gx) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n_trg; ++i) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int64_t j = 0; j < n_src; ++j) {
                if (skip_same_body && trg_body[i] == src_body[j])
                    continue;
                double d[3] = {x[3 * i] - y[3 * j], x[3 * i + 1] - y[3 * j + 1], x[3 * i + 2] - y[3 * j + 2]};
                double g[3];
                if (kind)
                    stokes_pair_grad(d, w + dim * i, s + dim * j, mu, g);
                else
                    laplace_pair_grad(d, w[i], s[j], g);
                acc[0] += g[0];
                acc[1] += g[1];
                acc[2] += g[2];
            }
            gx[3 * i] = acc[0];
            gx[3 * i + 1] = acc[1];
            gx[3 * i + 2] = acc[2];
        }
    }
    if (gy) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t j = 0; j < n_src; ++j) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int64_t i = 0; i < n_trg; ++i) {
                if (skip_same_body && trg_body[i] == src_body[j])
                    continue;
                double d[3] = {x[3 * i] - y[3 * j], x[3 * i + 1] - y[3 * j + 1], x[3 * i + 2] - y[3 * j + 2]};
                double g[3];
                if (kind)
                    stokes_pair_grad(d, w + dim * i, s + dim * j, mu, g);
                else
                    laplace_pair_grad(d, w[i], s[j], g);
                acc[0] -= g[0];
                acc[1] -= g[1];
                acc[2] -= g[2];
            }
            gy[3 * j] = acc[0];
            gy[3 * j + 1] = acc[1];
            gy[3 * j + 2] = acc[2];
        }
    }
}

int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

/*
 * Derived fields of the representation at arbitrary targets (same pair sets):
 *   field 0, Stokes pressure (Section 2.2):  p(x_i) = (1/(8 pi)) sum_j Pi(x_i - y_j) . f_j,
 *            with Pi(d) = 2 d / |d|^3;
 *   field 1, Stokes traction sigma(x_i) . n_i, with the stress of the Stokeslet
 *            (sigma = -p I + mu (grad u + grad u^T), eq. (traction)):
 *            sigma_ab(x_i) = -(3 / (4 pi)) sum_j d_a d_b (d . f_j) / |d|^5,
 *            and n_i the given unit vector at target i;
 *   field 2, Laplace gradient grad u(x_i) = -sum_j q_j d / (4 pi |d|^3).
 * d = x_i - y_j.  out is [n_trg] (field 0) or [n_trg][3].
 */
void oracle_p2p_field(int field, int64_t n_trg, const double *x, const int32_t *trg_body, const double *normal,
                      int64_t n_src, const double *y, const int32_t *src_body, const double *s,
                      int skip_same_body, double *out)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n_trg; ++i) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n_src; ++j) {
            if (skip_same_body && trg_body[i] == src_body[j])
                continue;
            double d[3] = {x[3 * i + 0] - y[3 * j + 0], x[3 * i + 1] - y[3 * j + 1], x[3 * i + 2] - y[3 * j + 2]};
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            if (field == 0) {
                const double *f = s + 3 * j;
                double Pi[3] = {2.0 * d[0] / (r * r2), 2.0 * d[1] / (r * r2), 2.0 * d[2] / (r * r2)};
                acc[0] += (Pi[0] * f[0] + Pi[1] * f[1] + Pi[2] * f[2]) / (8.0 * PI);
            } else if (field == 1) {
                const double *f = s + 3 * j;
                const double *n = normal + 3 * i;
                double sig[3][3];
                double df = d[0] * f[0] + d[1] * f[1] + d[2] * f[2];
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        sig[a][b] = -3.0 / (4.0 * PI) * d[a] * d[b] * df / (r2 * r2 * r);
                for (int a = 0; a < 3; ++a)
                    acc[a] += sig[a][0] * n[0] + sig[a][1] * n[1] + sig[a][2] * n[2];
            } else {
                for (int a = 0; a < 3; ++a)
                    acc[a] += -s[j] * d[a] / (4.0 * PI * r * r2);
            }
        }
        if (field == 0) {
            out[i] = acc[0];
        } else {
            out[3 * i + 0] = acc[0];
            out[3 * i + 1] = acc[1];
            out[3 * i + 2] = acc[2];
        }
    }
}
