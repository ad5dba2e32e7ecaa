// Derived fields of the MFS representation at arbitrary targets, gfx950.
//
// With d = x - y_j, r = |d|:
//   Stokes pressure (Section 2.2):  p(x) = (1/(8 pi)) sum_j Pi(d) . f_j,  Pi(d) = 2 d / r^3
//   Stokes traction sigma(x) . n with the stress of the Stokeslet sum
//     (sigma = -p I + mu (grad u + grad u^T), eq. (traction)):
//       sigma_ab(x) = -(3/(4 pi)) sum_j d_a d_b (d . f_j) / r^5   (independent of mu)
//   Laplace gradient:  grad u(x) = -(1/(4 pi)) sum_j q_j d / r^3
//
// The walk is the one of the pair sums: an item is 64 targets x a range of
// source bodies of one system, the four waves of the workgroup each take a
// contiguous quarter of every source body (wave-uniform loop, scalar-loaded
// sources), FP32 pairs on relative coordinates with FP64 accumulation per
// run of at most FLUSH sources (mixed) or FP64 throughout, and the waves'
// partial sums are added in wave order through LDS.  These fields are
// evaluated after a solve (surface traction, pressure, residual checks), not
// inside GMRES.
#include "device_math.h"
#include "mfs_internal.h"

namespace mfs {

namespace {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr int FLUSH = 64;

struct FieldArgs {
    const P2PItem *items;
    const double *centre;     // [n_body][3]
    const int32_t *trg_body;  // [n_trg]
    const int32_t *src_ptr;   // [n_body+1]
    const double *normal;     // [n_trg][3] (traction only)
    double *out;              // [n_trg][dim] or split slices of out_stride values
    int64_t out_stride;
    int skip_same;
    int accumulate;
};

template <bool MIXED, int FLD>
__global__ __launch_bounds__(BLOCK) void field_kernel(FieldArgs a, const void *__restrict__ trg_off_v,
                                                      const void *__restrict__ src_v) {
    typedef typename std::conditional<MIXED, float, double>::type R;
    constexpr int DIM = FLD == MFS_FIELD_PRESSURE ? 1 : 3;
    __shared__ double lds[(WAVES - 1) * 3 * 64];
    const P2PItem it = a.items[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = it.t0 + lane;
    const bool valid = i < it.t1;
    const int ii = valid ? i : it.t0;
    const int body = a.trg_body[ii];
    const double ct[3] = {a.centre[3 * body], a.centre[3 * body + 1], a.centre[3 * body + 2]};
    R xt[3];
    if (MIXED) {
        const float4 o = reinterpret_cast<const float4 *>(trg_off_v)[ii];
        xt[0] = o.x; xt[1] = o.y; xt[2] = o.z;
    } else {
        const double4 o = reinterpret_cast<const double4 *>(trg_off_v)[ii];
        xt[0] = (R)o.x; xt[1] = (R)o.y; xt[2] = (R)o.z;
    }
    R nv[3] = {R(0), R(0), R(0)};
    if (FLD == MFS_FIELD_TRACTION)
        for (int c = 0; c < 3; ++c) nv[c] = (R)a.normal[3 * (int64_t)ii + c];
    double acc[3] = {0.0, 0.0, 0.0};

    for (int b = it.b0; b < it.b1; ++b) {
        const bool use = valid && !(a.skip_same && body == b);
        if (!__any(use)) continue;
        R xr[3];
        for (int c = 0; c < 3; ++c) xr[c] = xt[c] + (R)(ct[c] - a.centre[3 * b + c]);
        const int s0 = a.src_ptr[b], s1 = a.src_ptr[b + 1];
        const int qn = (s1 - s0 + WAVES - 1) / WAVES;
        const int j0 = min(s0 + wv * qn, s1), j1 = min(j0 + qn, s1);
        for (int jb = j0; jb < j1; jb += FLUSH) {
            const int je = min(jb + FLUSH, j1);
            R p0 = 0, p1 = 0, p2 = 0;
#pragma unroll 2
            for (int j = jb; j < je; ++j) {
                R y0, y1, y2, f0 = 0, f1 = 0, f2 = 0, q = 0;
                if (FLD == MFS_FIELD_LAPLACE_GRADIENT) {
                    if (MIXED) {
                        const float4 sj = reinterpret_cast<const float4 *>(src_v)[j];
                        y0 = sj.x; y1 = sj.y; y2 = sj.z; q = sj.w;
                    } else {
                        const SrcL64 &sj = reinterpret_cast<const SrcL64 *>(src_v)[j];
                        y0 = sj.v[0]; y1 = sj.v[1]; y2 = sj.v[2]; q = sj.v[3];
                    }
                } else if (MIXED) {
                    const SrcS32 &sj = reinterpret_cast<const SrcS32 *>(src_v)[j];
                    y0 = sj.pos.x; y1 = sj.pos.y; y2 = sj.pos.z;
                    f0 = sj.str.x; f1 = sj.str.y; f2 = sj.str.z;
                } else {
                    const SrcS64 &sj = reinterpret_cast<const SrcS64 *>(src_v)[j];
                    y0 = sj.pos[0]; y1 = sj.pos[1]; y2 = sj.pos[2];
                    f0 = sj.str[0]; f1 = sj.str[1]; f2 = sj.str[2];
                }
                const R d0 = xr[0] - y0, d1 = xr[1] - y1, d2 = xr[2] - y2;
                const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
                R ri;
                if (MIXED) ri = __builtin_amdgcn_rsqf((float)r2);
                else ri = (R)rsqrt_f64((double)r2);
                const R ri2 = ri * ri;
                const R ri3 = ri * ri2;
                if (FLD == MFS_FIELD_PRESSURE) {
                    p0 += (d0 * f0 + d1 * f1 + d2 * f2) * ri3;
                } else if (FLD == MFS_FIELD_TRACTION) {
                    const R c = (d0 * nv[0] + d1 * nv[1] + d2 * nv[2]) * (d0 * f0 + d1 * f1 + d2 * f2) * ri3 * ri2;
                    p0 += c * d0;
                    p1 += c * d1;
                    p2 += c * d2;
                } else {
                    const R c = q * ri3;
                    p0 += c * d0;
                    p1 += c * d1;
                    p2 += c * d2;
                }
            }
            acc[0] += use ? (double)p0 : 0.0;
            acc[1] += use ? (double)p1 : 0.0;
            acc[2] += use ? (double)p2 : 0.0;
        }
    }
    // waves 1..3 hand their partial sums to wave 0, which adds them in wave order
    if (wv > 0)
        for (int c = 0; c < DIM; ++c) lds[((wv - 1) * 3 + c) * 64 + lane] = acc[c];
    __syncthreads();
    if (wv > 0) return;
    for (int w = 1; w < WAVES; ++w)
        for (int c = 0; c < DIM; ++c) acc[c] += lds[((w - 1) * 3 + c) * 64 + lane];
    if (!valid) return;
    const double scale = FLD == MFS_FIELD_PRESSURE ? 1.0 / (4.0 * PI)
                         : FLD == MFS_FIELD_TRACTION ? -3.0 / (4.0 * PI)
                                                     : -1.0 / (4.0 * PI);
    double *out = a.out + (int64_t)it.split * a.out_stride + DIM * (int64_t)i;
    for (int c = 0; c < DIM; ++c) {
        double v = scale * acc[c];
        if (a.accumulate) v += out[c];
        out[c] = v;
    }
}

__global__ void field_reduce_kernel(int64_t n, const double *__restrict__ partial, int64_t stride, int n_split,
                                    double *__restrict__ out, int accumulate) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double s = 0.0;
    for (int k = 0; k < n_split; ++k) s += partial[k * stride + v];
    if (accumulate) s += out[v];
    out[v] = s;
}

// Surface residual per test point.  Stokes: eps(x) = |u(x) - g(x)| / |g(x)| with g = v + omega x (x - c)
// from the body's rigid motion (eq. (residual)).  Laplace: the absolute error |u(x) - phi_k| against the
// body potential, the measure of the elastance convergence study (Sec. 4.1, Fig. f:elastconv(a)); a relative
// one would divide by potentials that may be near zero.
__global__ void residual_kernel(int64_t n, const int32_t *__restrict__ body, const int32_t *__restrict__ kind,
                                const int64_t *__restrict__ net_off, const double *__restrict__ off64,
                                const double *__restrict__ u, const int64_t *__restrict__ u_off,
                                const double *__restrict__ motion, double *__restrict__ eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int b = body[i];
    const double *m = motion + net_off[b];
    const double *ui = u + u_off[i];
    if (kind[b] == MFS_LAPLACE) {
        eps[i] = fabs(ui[0] - m[0]);
        return;
    }
    const double *d = off64 + 4 * i;
    const double g[3] = {m[0] + m[4] * d[2] - m[5] * d[1], m[1] + m[5] * d[0] - m[3] * d[2],
                         m[2] + m[3] * d[1] - m[4] * d[0]};
    const double e0 = ui[0] - g[0], e1 = ui[1] - g[1], e2 = ui[2] - g[2];
    eps[i] = sqrt(e0 * e0 + e1 * e1 + e2 * e2) / sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
}

template <bool MIXED>
void launch_field_kernel(int field, dim3 grid, const FieldArgs &a, const void *trg_off, const void *src,
                         hipStream_t s) {
    if (field == MFS_FIELD_PRESSURE)
        field_kernel<MIXED, MFS_FIELD_PRESSURE><<<grid, BLOCK, 0, s>>>(a, trg_off, src);
    else if (field == MFS_FIELD_TRACTION)
        field_kernel<MIXED, MFS_FIELD_TRACTION><<<grid, BLOCK, 0, s>>>(a, trg_off, src);
    else
        field_kernel<MIXED, MFS_FIELD_LAPLACE_GRADIENT><<<grid, BLOCK, 0, s>>>(a, trg_off, src);
}

}  // namespace

int launch_field(int field, const P2PPlan &pp, const P2PLaunch &L, const double *normal, int64_t n_trg,
                 hipStream_t s) {
    if (pp.items.empty()) return MFS_OK;
    if (pp.tpl != 1) return fail(MFS_EINVAL, "field sums take items of one target per lane");
    const int dim = field == MFS_FIELD_PRESSURE ? 1 : 3;
    FieldArgs a;
    a.items = pp.d_items.as<P2PItem>();
    a.centre = L.centre;
    a.trg_body = L.trg_body;
    a.src_ptr = L.src_ptr;
    a.normal = normal;
    a.skip_same = L.skip_same ? 1 : 0;
    const bool direct = pp.n_split == 1;
    a.out = direct ? L.out : L.partial;
    a.out_stride = dim * n_trg;
    a.accumulate = direct ? (L.accumulate ? 1 : 0) : 0;
    const void *src = field == MFS_FIELD_LAPLACE_GRADIENT ? L.srcL : L.srcS;
    const dim3 grid((unsigned)pp.items.size());
    if (L.prec == MFS_MIXED) launch_field_kernel<true>(field, grid, a, L.trg_off, src, s);
    else launch_field_kernel<false>(field, grid, a, L.trg_off, src, s);
    MFS_HIP_TRY(hipGetLastError());
    if (!direct) {
        const int64_t n = dim * n_trg;
        field_reduce_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, L.partial, n, pp.n_split, L.out,
                                                                       L.accumulate ? 1 : 0);
        MFS_HIP_TRY(hipGetLastError());
    }
    return MFS_OK;
}

int launch_residual(int64_t n, const int32_t *body, const int32_t *kind, const int64_t *net_off, const double *off64,
                    const double *u, const int64_t *u_off, const double *motion, double *eps, hipStream_t s) {
    if (n == 0) return MFS_OK;
    residual_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, body, kind, net_off, off64, u, u_off, motion, eps);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

}  // namespace mfs
