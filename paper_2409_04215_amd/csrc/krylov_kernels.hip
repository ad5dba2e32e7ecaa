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

// out[i] = sum_{n in chunk} V[i][n] w[n], i < nvec (one workgroup of 256 threads per chunk;
// thread t visits n = begin + t, begin + t + 256, ...)
__device__ __forceinline__ void chunk_dots(const VecChunk ch, const double *V, int64_t ldv, int nvec,
                                           const double *w, double *__restrict__ out, double (*sh)[DOT_GROUP]) {
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
        if (tid < ni) out[i0 + tid] = sh[0][tid] + sh[1][tid] + sh[2][tid] + sh[3][tid];
        __syncthreads();
    }
}

// sum_i V[i][n] cf[i], i < nvec, added in order of i; loads issued DOT_GROUP at a time
__device__ __forceinline__ double combine(const double *__restrict__ V, int64_t ldv, int nvec,
                                          const double *__restrict__ cf, int64_t n) {
    double acc = 0.0;
    int i = 0;
    for (; i + DOT_GROUP <= nvec; i += DOT_GROUP) {
        double v[DOT_GROUP];
#pragma unroll
        for (int q = 0; q < DOT_GROUP; ++q) v[q] = V[(int64_t)(i + q) * ldv + n];
#pragma unroll
        for (int q = 0; q < DOT_GROUP; ++q) acc += v[q] * cf[i + q];
    }
    for (; i < nvec; ++i) acc += V[(int64_t)i * ldv + n] * cf[i];
    return acc;
}

// partial[c][i] = sum_{n in chunk c} V[i][n] w[n], i < nvec
__global__ __launch_bounds__(256) void multi_dot_kernel(const VecChunk *__restrict__ chunks, const double *__restrict__ V,
                                                        int64_t ldv, int nvec, const double *__restrict__ w,
                                                        double *__restrict__ partial, int ld_partial) {
    __shared__ double sh[4][DOT_GROUP];
    chunk_dots(chunks[blockIdx.x], V, ldv, nvec, w, partial + (int64_t)blockIdx.x * ld_partial, sh);
}

// w[n] += sign * sum_i V[i][n] coef[sys(n)][i] (i < nvec), then on the updated chunk
// partial[c][i] = sum_n D[i][n] w[n] (i < ndot): an axpy and the next dot products in one pass.
// Each thread reads back only the w entries it wrote, so no barrier separates the two.
__global__ __launch_bounds__(256) void axpy_dot_kernel(const VecChunk *__restrict__ chunks, const double *__restrict__ V,
                                                       int64_t ldv, int nvec, const double *__restrict__ coef, int ld_coef,
                                                       double sign, double *w, const double *D, int64_t ldd, int ndot,
                                                       double *__restrict__ partial, int ld_partial) {
    __shared__ double sh[4][DOT_GROUP];
    const VecChunk ch = chunks[blockIdx.x];
    const double *cf = coef + (int64_t)ch.sys * ld_coef;
    for (int64_t n = ch.begin + threadIdx.x; n < ch.end; n += 256) w[n] += sign * combine(V, ldv, nvec, cf, n);
    chunk_dots(ch, D, ldd, ndot, w, partial + (int64_t)blockIdx.x * ld_partial, sh);
}

// sum over the chunks of system s of partial[c][i], by a workgroup of 256 threads: threads
// stride over the chunks, then a fixed-order tree reduction; the result is valid in thread 0
__device__ __forceinline__ double sys_sum(const int32_t *__restrict__ sys_chunk_ptr, const double *__restrict__ partial,
                                          int ld_partial, int i, int s, double *sh) {
    double acc = 0.0;
    for (int c = sys_chunk_ptr[s] + threadIdx.x; c < sys_chunk_ptr[s + 1]; c += 256)
        acc += partial[(int64_t)c * ld_partial + i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    return sh[0] + sh[1] + sh[2] + sh[3];
}

// out[s][i] = sum over chunks of system s of partial[c][i]; one block per (i, s)
__global__ __launch_bounds__(256) void reduce_sys_kernel(const int32_t *__restrict__ sys_chunk_ptr,
                                                         const double *__restrict__ partial, int ld_partial,
                                                         double *__restrict__ out, int ld_out) {
    __shared__ double sh[4];
    const int i = blockIdx.x, s = blockIdx.y;
    const double v = sys_sum(sys_chunk_ptr, partial, ld_partial, i, s, sh);
    if (threadIdx.x == 0) out[(int64_t)s * ld_out + i] = v;
}

// w[n] += sign * sum_i V[i][n] coef[sys(n)][i]
__global__ void multi_axpy_kernel(const VecChunk *__restrict__ chunks, const double *__restrict__ V, int64_t ldv, int nvec,
                                  const double *__restrict__ coef, int ld_coef, double sign, double *__restrict__ w) {
    const VecChunk ch = chunks[blockIdx.x];
    const double *cf = coef + (int64_t)ch.sys * ld_coef;
    for (int64_t n = ch.begin + threadIdx.x; n < ch.end; n += blockDim.x) w[n] += sign * combine(V, ldv, nvec, cf, n);
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

// ---------------------------------------------------------------------------
// GMRES least squares on the device, one thread per system
// ---------------------------------------------------------------------------
__global__ void givens_init_kernel(GivensState st) {
    const int sy = blockIdx.x * blockDim.x + threadIdx.x;
    if (sy >= st.n_sys) return;
    const double b = st.beta[sy];
    st.g[(int64_t)sy * (st.cap + 1)] = b;
    st.k[sy] = 0;
    st.est[sy] = b;
    st.scale[sy] = st.live[sy] ? 1.0 / b : 0.0;
}

// Column j of system sy (see givens_step_kernel); returns the status flags.
__device__ int givens_column(const GivensState &st, int j, int sy) {
    st.scale[sy] = 0.0;
    if (!st.live[sy]) return 0;
    const double *__restrict__ d0 = st.dots + (int64_t)sy * 2 * st.ldh;
    const double *__restrict__ d1 = d0 + st.ldh;
    const double *__restrict__ cs = st.cs + (int64_t)sy * st.cap;
    const double *__restrict__ sn = st.sn + (int64_t)sy * st.cap;
    double *__restrict__ Rj = st.R + (int64_t)sy * ((int64_t)st.cap * (st.cap + 1) / 2) + (int64_t)j * (j + 1) / 2;
    double *__restrict__ g = st.g + (int64_t)sy * (st.cap + 1);
    const double n2 = st.nrm2[sy];
    const double hn = isnan(n2) ? n2 : sqrt(fmax(0.0, n2));
    if (!isfinite(hn)) {
        st.live[sy] = 0;
        return 2;
    }
    double hi = d0[0] + d1[0];  // h_i as rotated so far
    for (int i = 0; i < j; ++i) {
        const double hnext = d0[i + 1] + d1[i + 1];
        Rj[i] = cs[i] * hi + sn[i] * hnext;
        hi = -sn[i] * hi + cs[i] * hnext;
    }
    const double rho = hypot(hi, hn);
    if (!(rho > 0.0)) {
        Rj[j] = 0.0;
        st.k[sy] = j;
        st.live[sy] = 0;
        return 0;
    }
    const double c = hi / rho, s = hn / rho;
    st.cs[(int64_t)sy * st.cap + j] = c;
    st.sn[(int64_t)sy * st.cap + j] = s;
    Rj[j] = rho;
    const double gj = g[j];
    g[j + 1] = -s * gj;
    g[j] = c * gj;
    st.k[sy] = j + 1;
    const double e = fabs(g[j + 1]);
    st.est[sy] = e;
    const bool go_on = !(e <= st.target[sy] || hn == 0.0);
    st.live[sy] = go_on;
    if (go_on) st.scale[sy] = 1.0 / hn;
    return go_on ? 1 : 0;
}

// Iteration j: column j of the Hessenberg matrix is h_i = (both CGS passes' coefficients)
// for i <= j and h_{j+1} = |w|.  The earlier rotations act on it in order, a new rotation
// zeroes h_{j+1}, and the rotated right-hand side g gives the residual estimate |g_{j+1}|.
// A system stops when that estimate reaches its target, when h_{j+1} = 0 (the Krylov space
// holds the solution), or at an exact breakdown (rho = 0: the solution lies in the first
// j columns).  A non-finite column stops the system and flags it.  Every system's estimate
// and flags go to the status block of the iteration.
// The last reduction of the iteration runs in the same launch, one workgroup per system:
// |w|^2 of system sy from the chunk partials (the same sum reduce_sys_kernel forms), then
// the step in thread 0.
__global__ __launch_bounds__(256) void norm_givens_kernel(GivensState st, const int32_t *__restrict__ sys_chunk_ptr,
                                                          const double *__restrict__ partial, int ld_partial,
                                                          double *nrm2, int j,  // aliases st.nrm2
                                                          double *__restrict__ status_est,
                                                          int32_t *__restrict__ status_flag) {
    __shared__ double sh[4];
    const int sy = blockIdx.x;
    const double v = sys_sum(sys_chunk_ptr, partial, ld_partial, 0, sy, sh);
    if (threadIdx.x != 0) return;
    nrm2[sy] = v;  // st.nrm2 points here: read back by this thread in givens_column
    const int flag = givens_column(st, j, sy);
    status_est[sy] = st.est[sy];
    status_flag[sy] = flag;
}

// y = R^-1 g over the first k columns (back substitution); coef[sy][i] = y_i for i < k,
// 0 for k <= i < nvec.
__global__ void givens_solve_kernel(GivensState st, double *__restrict__ coef, int ld_coef, int nvec) {
    const int sy = blockIdx.x * blockDim.x + threadIdx.x;
    if (sy >= st.n_sys) return;
    const int kk = st.k[sy];
    const double *__restrict__ R = st.R + (int64_t)sy * ((int64_t)st.cap * (st.cap + 1) / 2);
    const double *__restrict__ g = st.g + (int64_t)sy * (st.cap + 1);
    double *__restrict__ y = coef + (int64_t)sy * ld_coef;
    for (int i = kk; i < nvec; ++i) y[i] = 0.0;
    for (int i = kk - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < kk; ++c) t -= R[(int64_t)c * (c + 1) / 2 + i] * y[c];
        y[i] = t / R[(int64_t)i * (i + 1) / 2 + i];
    }
}

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

int launch_axpy_dot(int n_chunk, const VecChunk *chunks, const double *V, int64_t ldv, int nvec, const double *coef,
                    int ld_coef, double sign, double *w, const double *D, int64_t ldd, int ndot, double *partial,
                    int ld_partial, hipStream_t s) {
    if (n_chunk == 0) return MFS_OK;
    axpy_dot_kernel<<<n_chunk, 256, 0, s>>>(chunks, V, ldv, nvec, coef, ld_coef, sign, w, D, ldd, ndot, partial,
                                            ld_partial);
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

int launch_givens_init(const GivensState &st, hipStream_t s) {
    if (st.n_sys == 0) return MFS_OK;
    givens_init_kernel<<<(unsigned)((st.n_sys + 63) / 64), 64, 0, s>>>(st);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_givens_step(const GivensState &st, const int32_t *sys_chunk_ptr, const double *partial, int ld_partial,
                       double *nrm2, int j, double *status_est, int32_t *status_flag, hipStream_t s) {
    if (st.n_sys == 0) return MFS_OK;
    if (j < 0 || j >= st.cap) return fail(MFS_EINVAL, "internal: GMRES step beyond the Krylov capacity");
    if (nrm2 != st.nrm2) return fail(MFS_EINVAL, "internal: the step's norm buffer must be the Givens state's");
    norm_givens_kernel<<<(unsigned)st.n_sys, 256, 0, s>>>(st, sys_chunk_ptr, partial, ld_partial, nrm2, j, status_est,
                                                          status_flag);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_givens_solve(const GivensState &st, double *coef, int ld_coef, int nvec, hipStream_t s) {
    if (st.n_sys == 0) return MFS_OK;
    if (nvec > ld_coef || nvec > st.cap) return fail(MFS_EINVAL, "internal: GMRES solve beyond the Krylov capacity");
    givens_solve_kernel<<<(unsigned)((st.n_sys + 63) / 64), 64, 0, s>>>(st, coef, ld_coef, nvec);
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
