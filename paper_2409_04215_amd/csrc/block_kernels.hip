// One-body (block-diagonal) operators, gfx950.
//
//  * Pseudo-inverse blocks S_L^+ v = V Sigma^+ (U^T v), applied in two steps
//    and never formed (Section 2.3, eq. (pseudo)).  All bodies sharing a
//    factor are one GEMM: the columns are the bodies' vectors rotated into the
//    shape frame (Remark "congruent": lambda = R V Sigma^+ U^T R^T gamma).
//    GEMMs run on the matrix cores: v_mfma_f32_32x32x2_f32 (mixed) or
//    v_mfma_f64_16x16x4_f64 (FP64), one 32x32 output tile per wave loaded
//    straight into registers, one launch for every (factor, body-column)
//    tile of every shape.
//  * Projection (I - L): constants for Laplace (Section 3.1); rigid motions
//    L = K_N (K_N^T K_N)^{-1} K_N^T for Stokes (Section 3.2).  Never formed:
//    a 6-vector reduction w = K_N^T v, z = G^{-1} w, v - K_N z.  FP64.
//  * Completion strengths (eqs. (al0), (lambda01), (lambda02)), recovery of
//    phi / U (eqs. (vkal), (getU)), and setup assembly of
//    S_L = S^(kk)(I - L) + L_r in FP64 (Section 3.3).
#include "mfs_internal.h"

namespace mfs {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Grouped GEMM: C[:, col] = A_g * B[:, col] for every column of every group.
// A_g row-major (M x K, lda = K) in a factor pool; B and C columns are
// contiguous vectors at per-column element offsets.
//
// One wave computes one 32 x 32 output tile over a K range.  Fragments are
// loaded straight from global memory into registers (no LDS): the order in
// which the K index is visited is permuted per lane so that every lane reads
// contiguous runs of its own A row and B column (any bijection of K that A
// and B share leaves the product unchanged).
//  * f32, v_mfma_f32_32x32x2f32: lane l holds A[l%32][k] and B[k][l%32];
//    lanes 0-31 walk k in [k0, k0+32), lanes 32-63 in [k0+32, k0+64).
//  * f64, v_mfma_f64_16x16x4f64 (2 x 2 blocks of 16 x 16): lane l holds
//    A[l%16][k] and B[k][l%16]; lane group l/16 walks 16 consecutive k.
// A K range is split across waves when there are few output tiles; split
// slices land in a partial buffer that a second kernel sums in a fixed order.
// ---------------------------------------------------------------------------
constexpr int KT = 64;  // K per register tile

template <class T, int N>
__device__ __forceinline__ void load_run(const T *__restrict__ p, int k, int K, bool ok, bool vec, T (&v)[N]) {
    // v[t] = p[k + t] for k + t < K (else 0); p is a row or column start
    if (ok && vec && k + N <= K) {
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int t = 0; t < N; t += 4) {
                const float4 q = *reinterpret_cast<const float4 *>(p + k + t);
                v[t] = q.x; v[t + 1] = q.y; v[t + 2] = q.z; v[t + 3] = q.w;
            }
        } else {
#pragma unroll
            for (int t = 0; t < N; t += 2) {
                const double2 q = *reinterpret_cast<const double2 *>(p + k + t);
                v[t] = q.x; v[t + 1] = q.y;
            }
        }
    } else {
#pragma unroll
        for (int t = 0; t < N; ++t) v[t] = (ok && k + t < K) ? p[k + t] : T(0);
    }
}

template <class T>
__global__ __launch_bounds__(256) void gemm_kernel(int n_tiles, const GemmTile *__restrict__ tiles,
                                                   const GemmGroup *__restrict__ groups, const T *__restrict__ Apool,
                                                   const T *__restrict__ B, const int64_t *__restrict__ b_col_off,
                                                   T *__restrict__ C, const int64_t *__restrict__ c_col_off,
                                                   T *__restrict__ partial, int64_t part_col_stride,
                                                   int64_t part_split_stride, int vec_ok) {
    const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (task >= n_tiles) return;
    const GemmTile tl = tiles[task];
    const GemmGroup g = groups[tl.group];
    const T *A = Apool + g.a_off;
    const int lane = threadIdx.x & 63;
    const bool vec = vec_ok && (g.K % (sizeof(T) == 4 ? 4 : 2)) == 0;
    if constexpr (sizeof(T) == 4) {
        const int i = tl.m0 + (lane & 31), j = tl.n0 + (lane & 31), h = lane >> 5;
        const bool a_ok = i < g.M, b_ok = j < g.ncol;
        const T *arow = A + (int64_t)(a_ok ? i : 0) * g.K;
        const T *bcol = B + b_col_off[g.col_begin + (b_ok ? j : 0)];
        floatx16 acc = {};
        for (int k0 = tl.k0; k0 < tl.k1; k0 += KT) {
            float av[32], bv[32];
            load_run<float, 32>(arow, k0 + 32 * h, tl.k1, a_ok, vec, av);
            load_run<float, 32>(bcol, k0 + 32 * h, tl.k1, b_ok, vec, bv);
#pragma unroll
            for (int t = 0; t < 32; ++t) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[t], bv[t], acc, 0, 0, 0);
        }
        // D layout (32x32x2): lane l, reg r -> row 8*(r/4) + 4*(l/32) + r%4, col l%32
        const int col = tl.n0 + (lane & 31);
        if (col < g.ncol) {
            T *out = partial ? partial + tl.split * part_split_stride + (int64_t)(g.col_begin + col) * part_col_stride
                             : C + c_col_off[g.col_begin + col];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = tl.m0 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
                if (row < g.M) out[row] = acc[r];
            }
        }
    } else {
        const int q = lane >> 4, c16 = lane & 15;
        const T *arow[2];
        const T *bcol[2];
        bool a_ok[2], b_ok[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = tl.m0 + 16 * u + c16, j = tl.n0 + 16 * u + c16;
            a_ok[u] = i < g.M;
            b_ok[u] = j < g.ncol;
            arow[u] = A + (int64_t)(a_ok[u] ? i : 0) * g.K;
            bcol[u] = B + b_col_off[g.col_begin + (b_ok[u] ? j : 0)];
        }
        doublex4 acc[2][2] = {};
        for (int k0 = tl.k0; k0 < tl.k1; k0 += KT) {
            double av[2][16], bv[2][16];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                load_run<double, 16>(arow[u], k0 + 16 * q, tl.k1, a_ok[u], vec, av[u]);
                load_run<double, 16>(bcol[u], k0 + 16 * q, tl.k1, b_ok[u], vec, bv[u]);
            }
#pragma unroll
            for (int t = 0; t < 16; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int w = 0; w < 2; ++w)
                        acc[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t], bv[w][t], acc[u][w], 0, 0, 0);
        }
        // D layout (16x16x4 f64, measured on gfx950): lane l, reg r -> row l/16 + 4 r, col l%16
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int col = tl.n0 + 16 * w + c16;
            if (col >= g.ncol) continue;
            T *out = partial ? partial + tl.split * part_split_stride + (int64_t)(g.col_begin + col) * part_col_stride
                             : C + c_col_off[g.col_begin + col];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = tl.m0 + 16 * u + q + 4 * r;
                    if (row < g.M) out[row] = acc[u][w][r];
                }
        }
    }
}

// C[:, col] = sum over split slices (fixed order); blocks over (column, 256 rows), one thread per row
template <class T>
__global__ void gemm_reduce_kernel(const int32_t *__restrict__ col_group, const GemmGroup *__restrict__ groups,
                                   const T *__restrict__ partial, int64_t part_col_stride, int64_t part_split_stride,
                                   int n_split, T *__restrict__ C, const int64_t *__restrict__ c_col_off) {
    const int col = blockIdx.x;
    const int M = groups[col_group[col]].M;
    const int m = blockIdx.y * blockDim.x + threadIdx.x;
    if (m >= M) return;
    T s = 0;
    for (int sp = 0; sp < n_split; ++sp) s += partial[sp * part_split_stride + (int64_t)col * part_col_stride + m];
    C[c_col_off[col] + m] = s;
}

// ---------------------------------------------------------------------------
// Block reduction helper (256 threads)
// ---------------------------------------------------------------------------
template <int NV>
__device__ void block_sum(double (&v)[NV], double (*sh)[NV]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[q] = x;
    }
    if ((tid & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[tid >> 6][q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = sh[0][q] + sh[1][q] + sh[2][q] + sh[3][q];
    __syncthreads();
}

__device__ __forceinline__ void rot_apply(const double *R, const double *v, bool transpose, double *o) {
    if (!transpose) {
        for (int r = 0; r < 3; ++r) o[r] = R[3 * r] * v[0] + R[3 * r + 1] * v[1] + R[3 * r + 2] * v[2];
    } else {
        for (int r = 0; r < 3; ++r) o[r] = R[r] * v[0] + R[3 + r] * v[1] + R[6 + r] * v[2];
    }
}

// in (world frame fp64) -> out (shape frame, T); layout gamma (M points) or lambda (N points)
template <class T>
__global__ void rotate_in_kernel(BodyView bv, const double *__restrict__ in, T *__restrict__ out, int lam_layout) {
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = lam_layout ? bv.n_src[b] : bv.n_trg[b];
    const int64_t off = lam_layout ? bv.lam_off[b] : bv.gam_off[b];
    if (kind == MFS_LAPLACE) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) out[off + i] = (T)in[off + i];
        return;
    }
    double R[9];
    for (int q = 0; q < 9; ++q) R[q] = bv.rot[9 * b + q];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v[3] = {in[off + 3 * i], in[off + 3 * i + 1], in[off + 3 * i + 2]}, o[3];
        rot_apply(R, v, true, o);
        out[off + 3 * i] = (T)o[0];
        out[off + 3 * i + 1] = (T)o[1];
        out[off + 3 * i + 2] = (T)o[2];
    }
}

// shape frame T -> world fp64 (rotate with R), layout gamma or lambda
template <class T>
__global__ void rotate_out_kernel(BodyView bv, const T *__restrict__ in, double *__restrict__ out, int lam_layout) {
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = lam_layout ? bv.n_src[b] : bv.n_trg[b];
    const int64_t off = lam_layout ? bv.lam_off[b] : bv.gam_off[b];
    if (kind == MFS_LAPLACE) {
        for (int i = threadIdx.x; i < n; i += blockDim.x) out[off + i] = (double)in[off + i];
        return;
    }
    double R[9];
    for (int q = 0; q < 9; ++q) R[q] = bv.rot[9 * b + q];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        double v[3] = {(double)in[off + 3 * i], (double)in[off + 3 * i + 1], (double)in[off + 3 * i + 2]}, o[3];
        rot_apply(R, v, false, o);
        out[off + 3 * i] = o[0];
        out[off + 3 * i + 1] = o[1];
        out[off + 3 * i + 2] = o[2];
    }
}

__device__ __forceinline__ void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Strength of one pair-sum source record; the record array is chosen by the body kind.
__device__ __forceinline__ void write_src(void *srcS, void *srcL, int prec, int kind, int64_t row, const double *v) {
    if (kind == MFS_STOKES) {
        if (!srcS) return;
        if (prec == MFS_MIXED) {
            SrcS32 *p = reinterpret_cast<SrcS32 *>(srcS) + row;
            p->str = make_float4((float)v[0], (float)v[1], (float)v[2], 0.f);
        } else {
            SrcS64 *p = reinterpret_cast<SrcS64 *>(srcS) + row;
            p->str[0] = v[0];
            p->str[1] = v[1];
            p->str[2] = v[2];
        }
    } else {
        if (!srcL) return;
        if (prec == MFS_MIXED) reinterpret_cast<float4 *>(srcL)[row].w = (float)v[0];
        else reinterpret_cast<SrcL64 *>(srcL)[row].v[3] = v[0];
    }
}

// Projection of one body's strength vector, world frame, FP64.
// mode: 0 = (I - L) v ; also used to read the 6-vector / mean.
// Stokes: w = K_N^T v = [sum v_j; sum d_j x v_j]; z = G^{-1} w; out_j = v_j - (z_v + z_w x d_j)
template <class T>
__global__ __launch_bounds__(256) void project_kernel(BodyView bv, const T *__restrict__ lam, int rotate, int project,
                                                      double *__restrict__ out64, void *__restrict__ srcS,
                                                      void *__restrict__ srcL, int src_prec) {
    __shared__ double sh[4][6];
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    if (kind == MFS_LAPLACE) {
        double s[1] = {0.0};
        if (project) {
            for (int j = threadIdx.x; j < n; j += blockDim.x) s[0] += (double)lam[off + j];
            block_sum<1>(s, reinterpret_cast<double(*)[1]>(sh));
        }
        const double mean = project ? s[0] / n : 0.0;
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const double v = (double)lam[off + j] - mean;
            if (out64) out64[off + j] = v;
            write_src(srcS, srcL, src_prec, kind, row0 + j, &v);
        }
        return;
    }
    double R[9];
    for (int q = 0; q < 9; ++q) R[q] = bv.rot[9 * b + q];
    double z[6] = {0, 0, 0, 0, 0, 0};
    if (project) {
        double w[6] = {0, 0, 0, 0, 0, 0};
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            double v[3] = {(double)lam[off + 3 * j], (double)lam[off + 3 * j + 1], (double)lam[off + 3 * j + 2]};
            double vw[3];
            if (rotate) rot_apply(R, v, false, vw);
            else { vw[0] = v[0]; vw[1] = v[1]; vw[2] = v[2]; }
            const double *d = bv.src_off64 + 4 * (row0 + j);
            double c[3];
            cross3(d, vw, c);
            w[0] += vw[0]; w[1] += vw[1]; w[2] += vw[2];
            w[3] += c[0]; w[4] += c[1]; w[5] += c[2];
        }
        block_sum<6>(w, sh);
        const double *Gi = bv.gram_inv + 36 * b;
        for (int r = 0; r < 6; ++r) {
            double acc = 0.0;
            for (int c = 0; c < 6; ++c) acc += Gi[6 * r + c] * w[c];
            z[r] = acc;
        }
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double v[3] = {(double)lam[off + 3 * j], (double)lam[off + 3 * j + 1], (double)lam[off + 3 * j + 2]};
        double vw[3];
        if (rotate) rot_apply(R, v, false, vw);
        else { vw[0] = v[0]; vw[1] = v[1]; vw[2] = v[2]; }
        if (project) {
            const double *d = bv.src_off64 + 4 * (row0 + j);
            double c[3];
            cross3(z + 3, d, c);
            vw[0] -= z[0] + c[0];
            vw[1] -= z[1] + c[1];
            vw[2] -= z[2] + c[2];
        }
        if (out64) {
            out64[off + 3 * j] = vw[0];
            out64[off + 3 * j + 1] = vw[1];
            out64[off + 3 * j + 2] = vw[2];
        }
        write_src(srcS, srcL, src_prec, kind, row0 + j, vw);
    }
}

// Completion strengths s_0 (eqs. (al0); (lambda01), (lambda02)).
__global__ __launch_bounds__(256) void completion_kernel(BodyView bv, const double *__restrict__ net,
                                                         double *__restrict__ s0, void *__restrict__ srcS,
                                                         void *__restrict__ srcL, int src_prec) {
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    const double *nb = net + bv.net_off[b];
    if (kind == MFS_LAPLACE) {
        const double v = nb[0] / n;
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            if (s0) s0[off + j] = v;
            write_src(srcS, srcL, src_prec, kind, row0 + j, &v);
        }
        return;
    }
    const double *Gi = bv.gram_inv + 36 * b;
    double z[6];
    for (int r = 0; r < 6; ++r) {
        double acc = 0.0;
        for (int c = 0; c < 6; ++c) acc += Gi[6 * r + c] * nb[c];
        z[r] = acc;
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double *d = bv.src_off64 + 4 * (row0 + j);
        double c[3];
        cross3(z + 3, d, c);
        double v[3] = {z[0] + c[0], z[1] + c[1], z[2] + c[2]};
        if (s0) {
            s0[off + 3 * j] = v[0];
            s0[off + 3 * j + 1] = v[1];
            s0[off + 3 * j + 2] = v[2];
        }
        write_src(srcS, srcL, src_prec, kind, row0 + j, v);
    }
}

// Recovery: out = -mean(alpha) (Laplace) or -K_N^T lambda (Stokes); sigma = (I - L) lambda + s0.
// Dirichlet formulations (Section 2): out = sum(alpha) = q (eq. (qkgauss)) or
// K_N^T lambda = [f; t] (eq. (force_def)); sigma = lambda.
__global__ __launch_bounds__(256) void extract_kernel(BodyView bv, const double *__restrict__ lam,
                                                      const double *__restrict__ s0, double *__restrict__ out,
                                                      double *__restrict__ sigma) {
    __shared__ double sh[4][6];
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    if (bv.dirichlet && sigma)
        for (int j = threadIdx.x; j < (kind == MFS_LAPLACE ? n : 3 * n); j += blockDim.x) sigma[off + j] = lam[off + j];
    if (kind == MFS_LAPLACE) {
        double s[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += blockDim.x) s[0] += lam[off + j];
        block_sum<1>(s, reinterpret_cast<double(*)[1]>(sh));
        const double mean = s[0] / n;
        if (bv.dirichlet) {
            if (threadIdx.x == 0 && out) out[bv.net_off[b]] = s[0];
            return;
        }
        if (threadIdx.x == 0 && out) out[bv.net_off[b]] = -mean;
        if (sigma)
            for (int j = threadIdx.x; j < n; j += blockDim.x)
                sigma[off + j] = lam[off + j] - mean + (s0 ? s0[off + j] : 0.0);
        return;
    }
    double w[6] = {0, 0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double *v = lam + off + 3 * j;
        const double *d = bv.src_off64 + 4 * (row0 + j);
        double c[3];
        cross3(d, v, c);
        w[0] += v[0]; w[1] += v[1]; w[2] += v[2];
        w[3] += c[0]; w[4] += c[1]; w[5] += c[2];
    }
    block_sum<6>(w, sh);
    if (threadIdx.x == 0 && out)
        for (int q = 0; q < 6; ++q) out[bv.net_off[b] + q] = bv.dirichlet ? w[q] : -w[q];
    if (sigma && !bv.dirichlet) {
        const double *Gi = bv.gram_inv + 36 * b;
        double z[6];
        for (int r = 0; r < 6; ++r) {
            double acc = 0.0;
            for (int c = 0; c < 6; ++c) acc += Gi[6 * r + c] * w[c];
            z[r] = acc;
        }
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const double *v = lam + off + 3 * j;
            const double *d = bv.src_off64 + 4 * (row0 + j);
            double c[3];
            cross3(z + 3, d, c);
            for (int q = 0; q < 3; ++q)
                sigma[off + 3 * j + q] = v[q] - (z[q] + c[q]) + (s0 ? s0[off + 3 * j + q] : 0.0);
        }
    }
}

// dJ/dlambda from dJ/d(out): Stokes -K_N g (g = [gv; gw]); Laplace -(1/N) g.
__global__ void grad_lambda_kernel(BodyView bv, const double *__restrict__ gout, double *__restrict__ glam) {
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    const double *g = gout + bv.net_off[b];
    if (kind == MFS_LAPLACE) {
        for (int j = threadIdx.x; j < n; j += blockDim.x) glam[off + j] = -g[0] / n;
        return;
    }
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double *d = bv.src_off64 + 4 * (row0 + j);
        double c[3];
        cross3(g + 3, d, c);
        for (int q = 0; q < 3; ++q) glam[off + 3 * j + q] = -(g[q] + c[q]);
    }
}

__global__ void set_src_strength_kernel(BodyView bv, const double *__restrict__ str, void *__restrict__ srcS,
                                        void *__restrict__ srcL, int prec) {
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    const int dim = kind == MFS_STOKES ? 3 : 1;
    for (int j = threadIdx.x; j < n; j += blockDim.x) write_src(srcS, srcL, prec, kind, row0 + j, str + off + dim * j);
}

// grad_c[b] = sum over the body's targets of gt + sum over its sources of gs (fixed order)
__global__ __launch_bounds__(256) void body_grad_reduce_kernel(const int32_t *__restrict__ trg_ptr,
                                                               const int32_t *__restrict__ src_ptr,
                                                               const double *__restrict__ gt,
                                                               const double *__restrict__ gs,
                                                               double *__restrict__ grad_c) {
    __shared__ double sh[4][3];
    const int64_t b = blockIdx.x;
    double a[3] = {0, 0, 0};
    for (int i = trg_ptr[b] + threadIdx.x; i < trg_ptr[b + 1]; i += blockDim.x)
        for (int q = 0; q < 3; ++q) a[q] += gt[3 * (int64_t)i + q];
    for (int j = src_ptr[b] + threadIdx.x; j < src_ptr[b + 1]; j += blockDim.x)
        for (int q = 0; q < 3; ++q) a[q] += gs[3 * (int64_t)j + q];
    block_sum<3>(a, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) grad_c[3 * b + q] = a[q];
}

// ---------------------------------------------------------------------------
// Setup: S_L = S(I - L) + L_r in FP64, column-major (ld = dim*M), shape frame.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stokeslet64(const double *d, double mu, double G[3][3]) {
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = sqrt(r2);
    const double pref = 1.0 / (8.0 * PI * mu * r);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) G[a][c] = pref * ((a == c ? 1.0 : 0.0) + d[a] * d[c] / r2);
}

// K rows at point p: [I, (p)_x], with (p)_x = [[0, p2, -p1], [-p2, 0, p0], [p1, -p0, 0]]
__device__ __forceinline__ double Kentry(const double *p, int a, int q) {
    if (q < 3) return a == q ? 1.0 : 0.0;
    const int c = q - 3;
    const double X[3][3] = {{0.0, p[2], -p[1]}, {-p[2], 0.0, p[0]}, {p[1], -p[0], 0.0}};
    return X[a][c];
}

// Stokes step A: T_i = (S K_N)_i G^{-1} - K_M,i  (3 x 6 per target), work = [3M][6]
__global__ void sl_stokes_T_kernel(int M, int N, const double *__restrict__ trg, const double *__restrict__ src,
                                   const double *__restrict__ Gi, double mu, double *__restrict__ T) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    double SK[3][6] = {};
    const double *x = trg + 3 * i;
    for (int j = 0; j < N; ++j) {
        const double *y = src + 3 * j;
        double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        double G[3][3];
        stokeslet64(d, mu, G);
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < 6; ++q) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += G[a][c] * Kentry(y, c, q);
                SK[a][q] += s;
            }
    }
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 6; ++q) {
            double s = 0.0;
            for (int p = 0; p < 6; ++p) s += SK[a][p] * Gi[6 * p + q];
            T[(3 * i + a) * 6 + q] = s - Kentry(x, a, q);
        }
}

// Stokes step B: SL[row, col] = S[row, col] - sum_q T[row][q] K_N[col][q]
// (T null: the bare block S, for the Dirichlet formulations)
__global__ void sl_stokes_fill_kernel(int M, int N, const double *__restrict__ trg, const double *__restrict__ src,
                                      const double *__restrict__ T, double mu, double *__restrict__ SL) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // target point
    const int j = blockIdx.y;                              // source point
    if (i >= M) return;
    const double *x = trg + 3 * i;
    const double *y = src + 3 * j;
    double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
    double G[3][3];
    stokeslet64(d, mu, G);
    const int64_t ld = 3 * (int64_t)M;
    for (int c = 0; c < 3; ++c) {
        const int64_t col = 3 * j + c;
        for (int a = 0; a < 3; ++a) {
            double s = G[a][c];
            if (T)
                for (int q = 0; q < 6; ++q) s -= T[(3 * i + a) * 6 + q] * Kentry(y, c, q);
            SL[(3 * i + a) + col * ld] = s;
        }
    }
}

// Laplace: SL[i, j] = G_ij - mean_j' G_ij' + 1/N  (plain: the bare block G_ij)
__global__ void sl_laplace_kernel(int M, int N, const double *__restrict__ trg, const double *__restrict__ src,
                                  int plain, double *__restrict__ SL) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    const double *x = trg + 3 * i;
    double mean = 0.0;
    for (int j = 0; j < N; ++j) {
        const double *y = src + 3 * j;
        const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
        mean += 1.0 / (4.0 * PI * sqrt(d0 * d0 + d1 * d1 + d2 * d2));
    }
    mean /= N;
    for (int j = 0; j < N; ++j) {
        const double *y = src + 3 * j;
        const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
        const double g = 1.0 / (4.0 * PI * sqrt(d0 * d0 + d1 * d1 + d2 * d2));
        SL[i + (int64_t)j * M] = plain ? g : g - mean + 1.0 / N;
    }
}

// Dirichlet data at the collocation points of body b (gamma layout): the
// potential phi^(k) at every point (Section 2.1), or the rigid-body velocity
// v + omega x (x_i - c) (eq. (rbm); b = K_M U, Section 2.2).
__global__ __launch_bounds__(256) void dirichlet_rhs_kernel(BodyView bv, const double *__restrict__ data,
                                                            double *__restrict__ rhs) {
    const int64_t b = blockIdx.x;
    const int m = bv.n_trg[b];
    const int64_t off = bv.gam_off[b];
    const double *u = data + bv.net_off[b];
    if (bv.kind[b] == MFS_LAPLACE) {
        for (int i = threadIdx.x; i < m; i += blockDim.x) rhs[off + i] = u[0];
        return;
    }
    const int64_t row0 = bv.trg_row[b];
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double *d = bv.trg_off64 + 4 * (row0 + i);
        double c[3];
        cross3(u + 3, d, c);
        for (int q = 0; q < 3; ++q) rhs[off + 3 * i + q] = u[q] + c[q];
    }
}

// dst[r][c] (row-major rows x cols) = src(r, c) * rs[r] * cs[c], src(r,c) = transposed ? src[c*ld + r] : src[r*ld + c]
__global__ void make_factor_kernel(int rows, int cols, const double *__restrict__ src, int64_t ld, int transposed,
                                   const double *__restrict__ rs, const double *__restrict__ cs,
                                   double *__restrict__ d64, float *__restrict__ d32) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * cols) return;
    const int r = (int)(e / cols), c = (int)(e % cols);
    double v = transposed ? src[(int64_t)c * ld + r] : src[(int64_t)r * ld + c];
    if (rs) v *= rs[r];
    if (cs) v *= cs[c];
    d64[e] = v;
    d32[e] = (float)v;
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int launch_gemm_f32(const GemmLaunch &G, const float *Apool, const float *B, const int64_t *b_col_off, float *C,
                    const int64_t *c_col_off, float *partial, hipStream_t s) {
    if (G.n_tiles == 0) return MFS_OK;
    float *part = G.n_split > 1 ? partial : nullptr;
    gemm_kernel<float><<<(G.n_tiles + 3) / 4, 256, 0, s>>>(G.n_tiles, G.tiles, G.groups, Apool, B, b_col_off, C,
                                                          c_col_off, part, G.part_col_stride, G.part_split_stride, G.vec4);
    MFS_HIP_TRY(hipGetLastError());
    if (part) {
        gemm_reduce_kernel<float><<<dim3(G.n_cols, (unsigned)((G.part_col_stride + 255) / 256)), 256, 0, s>>>(
            G.col_group, G.groups, part, G.part_col_stride, G.part_split_stride, G.n_split, C, c_col_off);
        MFS_HIP_TRY(hipGetLastError());
    }
    return MFS_OK;
}

int launch_gemm_f64(const GemmLaunch &G, const double *Apool, const double *B, const int64_t *b_col_off, double *C,
                    const int64_t *c_col_off, double *partial, hipStream_t s) {
    if (G.n_tiles == 0) return MFS_OK;
    double *part = G.n_split > 1 ? partial : nullptr;
    gemm_kernel<double><<<(G.n_tiles + 3) / 4, 256, 0, s>>>(G.n_tiles, G.tiles, G.groups, Apool, B, b_col_off, C,
                                                            c_col_off, part, G.part_col_stride, G.part_split_stride, G.vec4);
    MFS_HIP_TRY(hipGetLastError());
    if (part) {
        gemm_reduce_kernel<double><<<dim3(G.n_cols, (unsigned)((G.part_col_stride + 255) / 256)), 256, 0, s>>>(
            G.col_group, G.groups, part, G.part_col_stride, G.part_split_stride, G.n_split, C, c_col_off);
        MFS_HIP_TRY(hipGetLastError());
    }
    return MFS_OK;
}

int launch_rotate_in(const BodyView &bv, const double *in, void *out, bool out_f32, bool lam_layout, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    if (out_f32) rotate_in_kernel<float><<<(unsigned)bv.n_body, 256, 0, s>>>(bv, in, (float *)out, lam_layout);
    else rotate_in_kernel<double><<<(unsigned)bv.n_body, 256, 0, s>>>(bv, in, (double *)out, lam_layout);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_rotate_out(const BodyView &bv, const void *in, bool in_f32, double *out, bool lam_layout, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    if (in_f32) rotate_out_kernel<float><<<(unsigned)bv.n_body, 256, 0, s>>>(bv, (const float *)in, out, lam_layout);
    else rotate_out_kernel<double><<<(unsigned)bv.n_body, 256, 0, s>>>(bv, (const double *)in, out, lam_layout);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_project(const BodyView &bv, const void *lam, bool lam_f32, bool rotate, bool project, double *out64,
                   void *srcS, void *srcL, int src_prec, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    if (lam_f32)
        project_kernel<float><<<(unsigned)bv.n_body, 256, 0, s>>>(bv, (const float *)lam, rotate, project, out64,
                                                                  srcS, srcL, src_prec);
    else
        project_kernel<double><<<(unsigned)bv.n_body, 256, 0, s>>>(bv, (const double *)lam, rotate, project, out64,
                                                                   srcS, srcL, src_prec);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_completion(const BodyView &bv, const double *net, double *s0, void *srcS, void *srcL, int src_prec,
                      hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    completion_kernel<<<(unsigned)bv.n_body, 256, 0, s>>>(bv, net, s0, srcS, srcL, src_prec);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_extract(const BodyView &bv, const double *lam, const double *s0, double *out, double *sigma, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    extract_kernel<<<(unsigned)bv.n_body, 256, 0, s>>>(bv, lam, s0, out, sigma);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_dirichlet_rhs(const BodyView &bv, const double *data, double *b, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    dirichlet_rhs_kernel<<<(unsigned)bv.n_body, 256, 0, s>>>(bv, data, b);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_grad_lambda(const BodyView &bv, const double *grad_out, double *glam, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    grad_lambda_kernel<<<(unsigned)bv.n_body, 256, 0, s>>>(bv, grad_out, glam);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_set_src_strength(const BodyView &bv, const double *str, void *srcS, void *srcL, int prec, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    set_src_strength_kernel<<<(unsigned)bv.n_body, 256, 0, s>>>(bv, str, srcS, srcL, prec);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_body_grad_reduce(int64_t n_body, const int32_t *trg_ptr, const int32_t *src_ptr, const double *gt,
                            const double *gs, double *grad_c, hipStream_t s) {
    if (n_body == 0) return MFS_OK;
    body_grad_reduce_kernel<<<(unsigned)n_body, 256, 0, s>>>(trg_ptr, src_ptr, gt, gs, grad_c);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_assemble_SL(int kind, int M, int N, const double *trg, const double *src, const double *gram_inv6,
                       double mu, bool plain, double *SL, double *work, hipStream_t s) {
    if (kind == MFS_LAPLACE) {
        sl_laplace_kernel<<<(M + 127) / 128, 128, 0, s>>>(M, N, trg, src, plain ? 1 : 0, SL);
        MFS_HIP_TRY(hipGetLastError());
        return MFS_OK;
    }
    if (!plain) {
        sl_stokes_T_kernel<<<(M + 63) / 64, 64, 0, s>>>(M, N, trg, src, gram_inv6, mu, work);
        MFS_HIP_TRY(hipGetLastError());
    }
    sl_stokes_fill_kernel<<<dim3((M + 127) / 128, N), 128, 0, s>>>(M, N, trg, src, plain ? nullptr : work, mu, SL);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_make_factor(int rows, int cols, const double *src, int64_t ld, bool transposed, const double *rs,
                       const double *cs, double *d64, float *d32, hipStream_t s) {
    const int64_t n = (int64_t)rows * cols;
    if (n == 0) return MFS_OK;
    make_factor_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rows, cols, src, ld, transposed ? 1 : 0, rs, cs,
                                                                  d64, d32);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

}  // namespace mfs
