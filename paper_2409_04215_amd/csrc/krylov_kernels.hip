// FP64 vector kernels for GMRES over a batch of independent systems.
//
// A Krylov vector is the concatenation of every system's gamma; it is cut
// into chunks that never straddle a system, so every reduction is a
// segmented one.  Dot products write one partial per chunk and a second
// kernel sums a system's chunks in a fixed order (deterministic results).
#include "mfs_internal.h"

namespace mfs {

namespace {

constexpr int DOT_GROUP = 8;

// partial[c][i] = sum_{n in chunk c} V[i][n] w[n], i < nvec
__global__ __launch_bounds__(256) void multi_dot_kernel(const VecChunk *__restrict__ chunks, const double *__restrict__ V,
                                                        int64_t ldv, int nvec, const double *__restrict__ w,
                                                        double *__restrict__ partial, int ld_partial) {
    __shared__ double sh[4][DOT_GROUP];
    const VecChunk ch = chunks[blockIdx.x];
    const int tid = threadIdx.x;
    for (int i0 = 0; i0 < nvec; i0 += DOT_GROUP) {
        double acc[DOT_GROUP];
#pragma unroll
        for (int q = 0; q < DOT_GROUP; ++q) acc[q] = 0.0;
        const int ni = min(DOT_GROUP, nvec - i0);
        for (int64_t n = ch.begin + tid; n < ch.end; n += 256) {
            const double wn = w[n];
#pragma unroll
            for (int q = 0; q < DOT_GROUP; ++q)
                if (q < ni) acc[q] += V[(int64_t)(i0 + q) * ldv + n] * wn;
        }
#pragma unroll
        for (int q = 0; q < DOT_GROUP; ++q) {
            double x = acc[q];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
            acc[q] = x;
        }
        if ((tid & 63) == 0)
#pragma unroll
            for (int q = 0; q < DOT_GROUP; ++q) sh[tid >> 6][q] = acc[q];
        __syncthreads();
        if (tid < ni) partial[(int64_t)blockIdx.x * ld_partial + i0 + tid] = sh[0][tid] + sh[1][tid] + sh[2][tid] + sh[3][tid];
        __syncthreads();
    }
}

// out[s][i] = sum over chunks of system s of partial[c][i]; one block per (i, s),
// threads stride over the chunks, then a fixed-order tree reduction.
__global__ __launch_bounds__(256) void reduce_sys_kernel(const int32_t *__restrict__ sys_chunk_ptr,
                                                         const double *__restrict__ partial, int ld_partial,
                                                         double *__restrict__ out, int ld_out) {
    __shared__ double sh[4];
    const int i = blockIdx.x, s = blockIdx.y;
    double acc = 0.0;
    for (int c = sys_chunk_ptr[s] + threadIdx.x; c < sys_chunk_ptr[s + 1]; c += 256)
        acc += partial[(int64_t)c * ld_partial + i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[(int64_t)s * ld_out + i] = sh[0] + sh[1] + sh[2] + sh[3];
}

// w[n] += sign * sum_i V[i][n] coef[sys(n)][i]
__global__ void multi_axpy_kernel(const VecChunk *__restrict__ chunks, const double *__restrict__ V, int64_t ldv, int nvec,
                                  const double *__restrict__ coef, int ld_coef, double sign, double *__restrict__ w) {
    const VecChunk ch = chunks[blockIdx.x];
    const double *cf = coef + (int64_t)ch.sys * ld_coef;
    for (int64_t n = ch.begin + threadIdx.x; n < ch.end; n += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < nvec; ++i) acc += V[(int64_t)i * ldv + n] * cf[i];
        w[n] += sign * acc;
    }
}

// out[n] = w[n] * scale[sys(n) * ld_scale]
__global__ void scale_sys_kernel(const VecChunk *__restrict__ chunks, const double *__restrict__ w,
                                 const double *__restrict__ scale, int ld_scale, double *__restrict__ out) {
    const VecChunk ch = chunks[blockIdx.x];
    const double f = scale[(int64_t)ch.sys * ld_scale];
    for (int64_t n = ch.begin + threadIdx.x; n < ch.end; n += blockDim.x) out[n] = w[n] * f;
}

__global__ void sub_kernel(int64_t n, const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = a[i] - b[i];
}

__global__ void add_kernel(int64_t n, const double *__restrict__ a, double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] += a[i];
}

__global__ void fill_kernel(int64_t n, double v, double *__restrict__ o) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) o[i] = v;
}

__global__ void finite_kernel(int64_t n, const double *__restrict__ x, int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(x[i])) atomicOr(flag, 1);
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

int launch_multi_dot(int n_chunk, const VecChunk *chunks, const double *V, int64_t ldv, int nvec, const double *w,
                     double *partial, int ld_partial, hipStream_t s) {
    if (n_chunk == 0 || nvec == 0) return MFS_OK;
    multi_dot_kernel<<<n_chunk, 256, 0, s>>>(chunks, V, ldv, nvec, w, partial, ld_partial);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_reduce_sys(int n_sys, const int32_t *sys_chunk_ptr, const double *partial, int ld_partial, int nval,
                      double *out, int ld_out, hipStream_t s) {
    if (n_sys == 0 || nval == 0) return MFS_OK;
    reduce_sys_kernel<<<dim3(nval, n_sys), 256, 0, s>>>(sys_chunk_ptr, partial, ld_partial, out, ld_out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_multi_axpy(int n_chunk, const VecChunk *chunks, const double *V, int64_t ldv, int nvec, const double *coef,
                      int ld_coef, double sign, double *w, hipStream_t s) {
    if (n_chunk == 0 || nvec == 0) return MFS_OK;
    multi_axpy_kernel<<<n_chunk, 256, 0, s>>>(chunks, V, ldv, nvec, coef, ld_coef, sign, w);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_scale_sys(int n_chunk, const VecChunk *chunks, const double *w, const double *scale, int ld_scale,
                     double *out, hipStream_t s) {
    if (n_chunk == 0) return MFS_OK;
    scale_sys_kernel<<<n_chunk, 256, 0, s>>>(chunks, w, scale, ld_scale, out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_sub(int64_t n, const double *a, const double *b, double *out, hipStream_t s) {
    if (n == 0) return MFS_OK;
    sub_kernel<<<nblk(n), 256, 0, s>>>(n, a, b, out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_add_inplace(int64_t n, const double *a, double *out, hipStream_t s) {
    if (n == 0) return MFS_OK;
    add_kernel<<<nblk(n), 256, 0, s>>>(n, a, out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_fill(int64_t n, double v, double *out, hipStream_t s) {
    if (n == 0) return MFS_OK;
    fill_kernel<<<nblk(n), 256, 0, s>>>(n, v, out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_check_finite(int64_t n, const double *x, int32_t *flag, hipStream_t s) {
    if (n == 0) return MFS_OK;
    finite_kernel<<<nblk(n), 256, 0, s>>>(n, x, flag);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

}  // namespace mfs
