// Batched FP64 QR factorisation of the one-body blocks on the GPU (gfx950).
//
// The pseudo-inverse of a full-column-rank m x n matrix A (m >= n) is
// A^+ = R^-1 Q^T with A = Q R (Q m x n with orthonormal columns, R n x n
// upper triangular): the same operator as V Sigma^-1 U^T from the SVD of
// Section 2.3, applied in the same two steps (Q^T, then R^-1).
//
// Blocked Householder QR (compact WY form).  The columns are taken in panels
// of NB = 16; the reflectors H_j = I - tau_j v_j v_j^T of one panel (v_j[j] = 1,
// stored below the diagonal of column j, R on and above it) multiply to
// H_k0 ... H_k0+kb-1 = I - V T V^T with T kb x kb upper triangular:
//   * panel_qr_kernel: one workgroup per matrix factors the panel column by
//     column (v_j, tau_j, R_jj, then H_j applied to the panel's later columns,
//     half a wave per column) and forms T from tau and the Gram matrix V^T V
//     (T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] (V^T v_j)[0:j]);
//   * wy_apply_kernel: the trailing columns C = A[k0:m, k0+kb:n] take
//     C <- (I - V T^T V^T) C, i.e. H_k0+kb-1 ... H_k0 applied at once, as
//     P = V^T C, W = T^T P, C -= V W, both products on the FP64 matrix cores
//     (v_mfma_f64_16x16x4f64); one workgroup per 16 columns.
// Q = H_0 H_1 ... H_{n-1} [I; 0] is accumulated panel by panel from the last
// one with the same kernel (C <- (I - V T V^T) C on rows k0..m-1 of columns
// k0..n-1; earlier columns of Q are still unit vectors there), and
// X = R^-1 comes from n independent triangular solves R x_i = e_i, one
// workgroup per column, with the running sums in LDS.
// Reductions add in a fixed order: results do not depend on timing.
#include <algorithm>

#include "mfs_internal.h"

namespace mfs {

namespace {

constexpr int FB = 256;   // threads per workgroup (inverse, ratio, WY update)
// Panel width.  16 columns made the QR of a 2400 x 1200 block faster than 32
// (panels 20.6 ms + updates 10.4 ms against 33 ms + 7.6 ms): the one-workgroup
// panel factorisation does half the work per column and the MFMA updates take
// the rest.  The kernels also build for NB = 32.
constexpr int NB = 16;
static_assert(NB == 16 || NB == 32, "the WY update's MFMA tiles cover 16 or 32 panel columns");
constexpr int PT = 32 * NB;  // threads of the panel kernel: half a wave per panel column
constexpr int PW = PT / 64;
constexpr int CT = 16;    // columns per workgroup of the WY update

typedef double doublex4 __attribute__((ext_vector_type(4)));

// sum over the workgroup in a fixed order (wave shuffles, then the waves in order)
template <int NW>
__device__ double block_sum_fixed(double x, double *sh) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// One panel (columns k0 .. k0+kb-1, rows k0 .. m-1) of every matrix; T of the panel to
// Tp[b][NB][NB] (row-major, zero outside the leading kb x kb upper triangle).
// Step j (column c = k0 + j): the norm of the column below the diagonal (all threads,
// fixed-order block sum), v_j and tau_j, then one pass over the panel's other columns:
// wave w owns columns 2w and 2w+1, lane l column 2w + l/32 and rows c+1 + l%32 + 32 i,
// so a column's partial sums are added by a 32-lane butterfly inside the wave (every lane
// gets the sum) and the same lanes apply H_j to that column without a barrier.  The same
// pass gives the Gram entries G[i][j] = v_i . v_j of the earlier columns (v_j is 1 at row
// c and zero above), from which T follows:
// T_jj = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j].
__global__ __launch_bounds__(PT) void panel_qr_kernel(double *__restrict__ A, int m, int lda, int64_t stride, int k0,
                                                      int kb, double *__restrict__ tau, int n, double *__restrict__ Tp) {
    __shared__ double sh[PW];
    __shared__ double G[NB][NB + 1];
    __shared__ double Ts[NB][NB + 1];
    __shared__ double tl[NB];
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int q = 2 * wave + (lane >> 5), g = lane & 31;  // this lane's panel column and row phase
    double *a = A + (int64_t)b * stride;
    double *xq = a + (int64_t)(k0 + q) * lda;  // dereferenced only for q < kb
    for (int j = 0; j < kb; ++j) {
        const int c = k0 + j;
        double *col = a + (int64_t)c * lda;
        const double alpha = col[c];  // read before the reduction's barriers: thread 0 overwrites it below
        double ss = 0.0;
        for (int r = c + 1 + t; r < m; r += PT) ss += col[r] * col[r];
        ss = block_sum_fixed<PW>(ss, sh);
        double tj = 0.0, scal = 1.0;  // nothing below the diagonal: H_j = I, R_jj = A_jj
        if (ss != 0.0) {
            const double nrm = sqrt(alpha * alpha + ss);
            const double beta = alpha >= 0.0 ? -nrm : nrm;  // no cancellation in alpha - beta
            scal = 1.0 / (alpha - beta);
            tj = (beta - alpha) / beta;
            for (int r = c + 1 + t; r < m; r += PT) col[r] *= scal;
            if (t == 0) col[c] = beta;
        }
        if (t == 0) {
            tau[(int64_t)b * n + c] = tj;
            tl[j] = tj;
        }
        __syncthreads();  // v_j in place
        if (q < kb && q != j) {
            double d = 0.0;
            int r = c + 1 + g;
            for (; r + 96 < m; r += 128) {  // four rows in flight per lane
                const double v0 = col[r], v1 = col[r + 32], v2 = col[r + 64], v3 = col[r + 96];
                const double x0 = xq[r], x1 = xq[r + 32], x2 = xq[r + 64], x3 = xq[r + 96];
                d += v0 * x0;
                d += v1 * x1;
                d += v2 * x2;
                d += v3 * x3;
            }
            for (; r < m; r += 32) d += col[r] * xq[r];
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
            const double xc = xq[c];
            if (q < j) {
                if (g == 0) G[q][j] = d + xc;  // v_q . v_j
            } else if (tj != 0.0) {
                const double w = (d + xc) * tj;
                for (int rr = c + 1 + g; rr < m; rr += 32) xq[rr] -= w * col[rr];
                if (g == 0) xq[c] = xc - w;
            }
        }
        __syncthreads();
    }
    // T column by column in wave 0: lane i owns row i, so it reads only its own earlier entries
    if (wave == 0 && lane < NB) {
        const int i = lane;
        for (int j = 0; j < NB; ++j) {
            double v = 0.0;
            if (j < kb) {
                if (i < j) {
                    double s = 0.0;
                    for (int l = i; l < j; ++l) s += Ts[i][l] * G[l][j];
                    v = -tl[j] * s;
                } else if (i == j) {
                    v = tl[j];
                }
            }
            Ts[i][j] = v;
        }
    }
    __syncthreads();
    double *T = Tp + (int64_t)b * NB * NB;
    for (int e = t; e < NB * NB; e += PT) T[e] = Ts[e / NB][e % NB];
}

// V[r][i] of the panel at k0 (unit lower trapezoidal, zero past kb columns or m rows)
__device__ __forceinline__ double panel_v(const double *__restrict__ v, int lda, int m, int k0, int kb, int r, int i) {
    if (i >= kb || r >= m) return 0.0;
    const int d = k0 + i;
    if (r < d) return 0.0;
    if (r == d) return 1.0;
    return v[(int64_t)d * lda + r];
}

// C[k0:m, c0:c1] <- (I - V op(T) V^T) C[k0:m, c0:c1] with V, T of the panel at k0;
// op(T) = T^T (TRANS: the QR's trailing update) or T (accumulating Q).
// Grid (column tiles of CT, batch); four waves.
//  1. P = V^T C (NB x CT): each wave sums a quarter of the rows in steps of 16;
//     MFMA A = V^T (lane l: V[r][k0 + l%16], and V[r][k0 + 16 + l%16] in a second
//     accumulator when NB = 32), B = C (lane l: C[r][col l%16]),
//     the k slot l/16 of MFMA t standing for row r = r0 + 4 (l/16) + t in both;
//     D layout (16x16x4 f64): lane l, reg q -> row l/16 + 4 q, col l%16.
//  2. The four partial P added in wave order, W = op(T) P in LDS.
//  3. C -= V W by 16-row blocks as D^T = W^T V^T (16 columns x 16 rows): lane l gives
//     W[k][l%16] and V[r0 + l%16][k0 + k] for k = 4 t + l/16, and holds C rows
//     r0 + l%16 of columns l/16 + 4 q: 16 consecutive rows of one column per
//     16 lanes, so the read-modify-write of C is coalesced.
template <bool TRANS>
__global__ __launch_bounds__(FB) void wy_apply_kernel(const double *__restrict__ V, int m, int lda, int64_t stride_v,
                                                      int k0, int kb, const double *__restrict__ Tp,
                                                      double *__restrict__ C, int ldc, int64_t stride_c, int c0,
                                                      int c1) {
    __shared__ double Pw[4][NB][CT];
    __shared__ double Ps[NB][CT];
    __shared__ double Wl[NB][CT];
    __shared__ double Ts[NB][NB + 1];
    const int b = blockIdx.y, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int q = lane >> 4, c16 = lane & 15;
    const int cbase = c0 + (int)blockIdx.x * CT;
    const double *v = V + (int64_t)b * stride_v;
    double *cm = C + (int64_t)b * stride_c;
    const double *T = Tp + (int64_t)b * NB * NB;
    for (int e = t; e < NB * NB; e += FB) Ts[e / NB][e % NB] = T[e];

    // 1. P = V^T C
    const int col = cbase + c16;
    const bool cok = col < c1;
    const double *ccol = cm + (int64_t)(cok ? col : c0) * ldc;
    doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    for (int r0 = k0 + 16 * wave; r0 < m; r0 += 64) {
        const int rb = r0 + 4 * q;
        double cv[4], va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = rb + u;
            cv[u] = (cok && r < m) ? ccol[r] : 0.0;
            va[u] = panel_v(v, lda, m, k0, kb, r, c16);
            if constexpr (NB == 32) vb[u] = panel_v(v, lda, m, k0, kb, r, 16 + c16);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], cv[u], acc0, 0, 0, 0);
            if constexpr (NB == 32) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(vb[u], cv[u], acc1, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Pw[wave][q + 4 * r][c16] = acc0[r];
        if constexpr (NB == 32) Pw[wave][16 + q + 4 * r][c16] = acc1[r];
    }
    __syncthreads();
    // 2. P summed over the waves in order, W = op(T) P
    for (int e = t; e < NB * CT; e += FB) {
        const int i = e / CT, j = e % CT;
        Ps[i][j] = ((Pw[0][i][j] + Pw[1][i][j]) + Pw[2][i][j]) + Pw[3][i][j];
    }
    __syncthreads();
    for (int e = t; e < NB * CT; e += FB) {
        const int i = e / CT, j = e % CT;
        double s = 0.0;
        if (TRANS) {
            for (int l = 0; l <= i; ++l) s += Ts[l][i] * Ps[l][j];  // (T^T)[i][l] = T[l][i], l <= i
        } else {
            for (int l = i; l < NB; ++l) s += Ts[i][l] * Ps[l][j];
        }
        Wl[i][j] = s;
    }
    __syncthreads();
    // 3. C -= V W
    for (int r0 = k0 + 16 * wave; r0 < m; r0 += 64) {
        const int r = r0 + c16;
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < NB / 4; ++u) {
            const int k = 4 * u + q;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Wl[k][c16], panel_v(v, lda, m, k0, kb, r, k), acc, 0, 0, 0);
        }
        if (r < m) {
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) {
                const int cc = cbase + q + 4 * rr;
                if (cc < c1) cm[(int64_t)cc * ldc + r] -= acc[rr];
            }
        }
    }
}

// Q = [I_n; 0] (column-major m x n, leading dimension m)
__global__ void identity_kernel(double *__restrict__ Q, int m, int n, int64_t stride, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t b = e / ((int64_t)m * n), q = e % ((int64_t)m * n);
    const int c = (int)(q / m), r = (int)(q % m);
    Q[b * stride + q] = r == c ? 1.0 : 0.0;
}

// X[:, i] = R^-1 e_i (column-major, upper triangular): x_k = (delta_ik - s_k) / R_kk for k = i..0,
// where s_k = sum_{l > k} R_kl x_l is accumulated column by column in LDS as the x_l appear.
// colsq[b][0][i] = sum_r R_ri^2 and colsq[b][1][i] = sum_r X_ri^2 for the norms of qr_ratio_kernel.
__global__ __launch_bounds__(FB) void upper_inverse_kernel(const double *__restrict__ R, int n, int ldr, int64_t stride_r,
                                                            double *__restrict__ X, int ldx, int64_t stride_x,
                                                            double *__restrict__ colsq) {
    extern __shared__ double s[];  // [n]
    __shared__ double xk_sh;
    __shared__ double sh[FB / 64];
    const int i = blockIdx.x, b = blockIdx.y;
    const double *Rb = R + (int64_t)b * stride_r;
    double *x = X + (int64_t)b * stride_x + (int64_t)i * ldx;
    for (int r = threadIdx.x; r <= i; r += FB) s[r] = 0.0;
    for (int r = i + 1 + threadIdx.x; r < n; r += FB) x[r] = 0.0;
    for (int k = i; k >= 0; --k) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const double xk = ((k == i) ? 1.0 : -s[k]) / Rb[(int64_t)k * ldr + k];
            x[k] = xk;
            xk_sh = xk;
        }
        __syncthreads();
        const double xk = xk_sh;
        const double *rk = Rb + (int64_t)k * ldr;  // column k of R, rows 0..k-1
        for (int r = threadIdx.x; r < k; r += FB) s[r] += rk[r] * xk;
    }
    __syncthreads();  // x[0..i] written by thread 0
    const double *ri = Rb + (int64_t)i * ldr;
    double sr = 0.0, sx = 0.0;
    for (int r = threadIdx.x; r <= i; r += FB) {
        sr += ri[r] * ri[r];
        sx += x[r] * x[r];
    }
    sr = block_sum_fixed<FB / 64>(sr, sh);
    sx = block_sum_fixed<FB / 64>(sx, sh);
    if (threadIdx.x == 0) {
        colsq[(int64_t)b * 2 * n + i] = sr;
        colsq[(int64_t)b * 2 * n + n + i] = sx;
    }
}

// ratio[b] = 1 / (||R||_F ||R^-1||_F), a lower bound of sigma_min / sigma_max
__global__ __launch_bounds__(FB) void qr_ratio_kernel(int n, const double *__restrict__ colsq, double *__restrict__ ratio) {
    __shared__ double sh[FB / 64];
    const int b = blockIdx.x;
    const double *c = colsq + (int64_t)b * 2 * n;
    double sr = 0.0, sx = 0.0;
    for (int i = threadIdx.x; i < n; i += FB) {
        sr += c[i];
        sx += c[n + i];
    }
    sr = block_sum_fixed<FB / 64>(sr, sh);
    sx = block_sum_fixed<FB / 64>(sx, sh);
    if (threadIdx.x == 0) ratio[b] = 1.0 / sqrt(sr * sx);
}

}  // namespace

size_t qr_scratch_doubles(int batch, int n) {
    const size_t panels = (size_t)(n + NB - 1) / NB;
    return (size_t)batch * n * 3 + panels * (size_t)batch * NB * NB;
}

int qr_inverse_batched(int batch, double *A, int m, int n, int64_t stride_a, double *Q, int64_t stride_q, double *X,
                       int64_t stride_x, double *scratch, double *ratio, hipStream_t s) {
    if (batch <= 0 || n <= 0) return MFS_OK;
    if (m < n) return fail(MFS_EINVAL, "QR factorisation needs rows >= columns");
    if ((size_t)n * sizeof(double) > 64 * 1024) return fail(MFS_EINVAL, "QR factorisation supports at most 8192 columns");
    if (batch > 65535) return fail(MFS_EINVAL, "QR factorisation: at most 65535 matrices per batch");
    double *tau = scratch;
    double *colsq = scratch + (size_t)batch * n;      // [batch][2][n]
    double *Tall = scratch + (size_t)batch * n * 3;  // T of panel p: Tall + p * batch * NB * NB
    const int panels = (n + NB - 1) / NB;
    for (int p = 0; p < panels; ++p) {
        const int k0 = p * NB, kb = std::min(NB, n - k0);
        double *Tp = Tall + (size_t)p * batch * NB * NB;
        panel_qr_kernel<<<batch, PT, 0, s>>>(A, m, m, stride_a, k0, kb, tau, n, Tp);
        if (k0 + kb < n)
            wy_apply_kernel<true><<<dim3((n - k0 - kb + CT - 1) / CT, batch), FB, 0, s>>>(
                A, m, m, stride_a, k0, kb, Tp, A, m, stride_a, k0 + kb, n);
    }
    MFS_HIP_TRY(hipGetLastError());
    const int64_t total = (int64_t)batch * m * n;
    identity_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(Q, m, n, stride_q, total);
    for (int p = panels - 1; p >= 0; --p) {
        const int k0 = p * NB, kb = std::min(NB, n - k0);
        wy_apply_kernel<false><<<dim3((n - k0 + CT - 1) / CT, batch), FB, 0, s>>>(
            A, m, m, stride_a, k0, kb, Tall + (size_t)p * batch * NB * NB, Q, m, stride_q, k0, n);
    }
    MFS_HIP_TRY(hipGetLastError());
    upper_inverse_kernel<<<dim3(n, batch), FB, (size_t)n * sizeof(double), s>>>(A, n, m, stride_a, X, n, stride_x,
                                                                               colsq);
    qr_ratio_kernel<<<batch, FB, 0, s>>>(n, colsq, ratio);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

}  // namespace mfs
