// Batched FP64 QR factorisation of the one-body blocks on the GPU (gfx950).
//
// The pseudo-inverse of a full-column-rank m x n matrix A (m >= n) is
// A^+ = R^-1 Q^T with A = Q R (Q m x n with orthonormal columns, R n x n
// upper triangular): the same operator as V Sigma^-1 U^T from the SVD of
// Section 2.3, applied in the same two steps (Q^T, then R^-1).
//
// Householder QR, one reflector at a time (H_j = I - tau_j v_j v_j^T with
// v_j[j] = 1, stored below the diagonal of column j, R on and above it):
//   * householder_vec_kernel: one workgroup per matrix forms v_j, tau_j and
//     R_jj from column j (the sign of beta opposite to A_jj, so no
//     cancellation);
//   * householder_apply_kernel: one workgroup per (column, matrix) applies
//     H_j to a column of the trailing matrix (QR) or of Q (accumulation).
// Each step is a rank-one (level-2) update, bound by memory traffic; the
// matrices of one batch share every launch.
// Q = H_0 H_1 ... H_{n-1} [I; 0] is accumulated backwards, and
// X = R^-1 comes from n independent triangular solves R x_i = e_i, one
// workgroup per column, with the running sums in LDS.
// Reductions add in a fixed order: results do not depend on timing.
#include "mfs_internal.h"

namespace mfs {

namespace {

constexpr int FB = 256;  // threads per workgroup

// sum over the workgroup in a fixed order (wave shuffles, then the four waves in order)
__device__ double block_sum_fixed(double x, double *sh) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    const double t = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return t;
}

__global__ __launch_bounds__(FB) void householder_vec_kernel(double *__restrict__ A, int m, int n, int lda,
                                                               int64_t stride, int j, double *__restrict__ tau) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    double *a = A + (int64_t)b * stride + (int64_t)j * lda;
    const double alpha = a[j];  // read before the reduction's barriers: thread 0 overwrites it below
    double ss = 0.0;
    for (int r = j + 1 + threadIdx.x; r < m; r += FB) ss += a[r] * a[r];
    ss = block_sum_fixed(ss, sh);
    if (ss == 0.0) {  // nothing below the diagonal: H_j = I, R_jj = A_jj
        if (threadIdx.x == 0) tau[(int64_t)b * n + j] = 0.0;
        return;
    }
    const double norm = sqrt(alpha * alpha + ss);
    const double beta = alpha >= 0.0 ? -norm : norm;
    const double scal = 1.0 / (alpha - beta);
    for (int r = j + 1 + threadIdx.x; r < m; r += FB) a[r] *= scal;
    if (threadIdx.x == 0) {
        a[j] = beta;
        tau[(int64_t)b * n + j] = (beta - alpha) / beta;
    }
}

// C[j:m, c] -= tau_j v_j (v_j . C[j:m, c]) for c in [c0, c0 + gridDim.x)
__global__ __launch_bounds__(FB) void householder_apply_kernel(const double *__restrict__ V, int m, int n, int ldv,
                                                                int64_t stride_v, const double *__restrict__ tau, int j,
                                                                double *__restrict__ C, int ldc, int64_t stride_c,
                                                                int c0) {
    __shared__ double sh[4];
    const int b = blockIdx.y;
    const double t = tau[(int64_t)b * n + j];
    if (t == 0.0) return;
    const double *v = V + (int64_t)b * stride_v + (int64_t)j * ldv;
    double *col = C + (int64_t)b * stride_c + (int64_t)(c0 + blockIdx.x) * ldc;
    const double cj = col[j];  // read before the reduction's barriers: thread 0 overwrites it below
    double w = 0.0;
    for (int r = j + 1 + threadIdx.x; r < m; r += FB) w += v[r] * col[r];
    w = (block_sum_fixed(w, sh) + cj) * t;
    if (threadIdx.x == 0) col[j] -= w;
    for (int r = j + 1 + threadIdx.x; r < m; r += FB) col[r] -= w * v[r];
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
__global__ __launch_bounds__(FB) void upper_inverse_kernel(const double *__restrict__ R, int n, int ldr, int64_t stride_r,
                                                            double *__restrict__ X, int ldx, int64_t stride_x) {
    extern __shared__ double s[];  // [n]
    __shared__ double xk_sh;
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
}

// ratio[b] = 1 / (||R||_F ||R^-1||_F), a lower bound of sigma_min / sigma_max
__global__ __launch_bounds__(FB) void qr_ratio_kernel(const double *__restrict__ R, int n, int ldr, int64_t stride_r,
                                                       const double *__restrict__ X, int ldx, int64_t stride_x,
                                                       double *__restrict__ ratio) {
    __shared__ double sh[4];
    const int b = blockIdx.x;
    double sr = 0.0, sx = 0.0;
    for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += FB) {
        const int c = (int)(e / n), r = (int)(e % n);
        if (r > c) continue;
        const double a = R[(int64_t)b * stride_r + (int64_t)c * ldr + r];
        const double y = X[(int64_t)b * stride_x + (int64_t)c * ldx + r];
        sr += a * a;
        sx += y * y;
    }
    sr = block_sum_fixed(sr, sh);
    sx = block_sum_fixed(sx, sh);
    if (threadIdx.x == 0) ratio[b] = 1.0 / sqrt(sr * sx);
}

}  // namespace

int qr_inverse_batched(int batch, double *A, int m, int n, int64_t stride_a, double *Q, int64_t stride_q, double *X,
                       int64_t stride_x, double *tau, double *ratio, hipStream_t s) {
    if (batch <= 0 || n <= 0) return MFS_OK;
    if (m < n) return fail(MFS_EINVAL, "QR factorisation needs rows >= columns");
    if ((size_t)n * sizeof(double) > 64 * 1024) return fail(MFS_EINVAL, "QR factorisation supports at most 8192 columns");
    if (batch > 65535) return fail(MFS_EINVAL, "QR factorisation: at most 65535 matrices per batch");
    for (int j = 0; j < n; ++j) {
        householder_vec_kernel<<<batch, FB, 0, s>>>(A, m, n, m, stride_a, j, tau);
        if (j + 1 < n)
            householder_apply_kernel<<<dim3(n - j - 1, batch), FB, 0, s>>>(A, m, n, m, stride_a, tau, j, A, m, stride_a,
                                                                          j + 1);
    }
    MFS_HIP_TRY(hipGetLastError());
    const int64_t total = (int64_t)batch * m * n;
    identity_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(Q, m, n, stride_q, total);
    for (int j = n - 1; j >= 0; --j)
        householder_apply_kernel<<<dim3(n - j, batch), FB, 0, s>>>(A, m, n, m, stride_a, tau, j, Q, m, stride_q, j);
    MFS_HIP_TRY(hipGetLastError());
    upper_inverse_kernel<<<dim3(n, batch), FB, (size_t)n * sizeof(double), s>>>(A, n, m, stride_a, X, n, stride_x);
    qr_ratio_kernel<<<batch, FB, 0, s>>>(A, n, m, stride_a, X, n, stride_x, ratio);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

}  // namespace mfs
