// One-body (block-diagonal) operators, gfx950.
//
//  * Pseudo-inverse blocks S_L^+ v = V Sigma^+ (U^T v), applied in two steps
//    and never formed (Section 2.3, eq. (pseudo)).  All bodies sharing a
//    factor are one GEMM: the columns are the bodies' vectors rotated into the
//    shape frame (Remark "congruent": lambda = R V Sigma^+ U^T R^T gamma).
//    GEMMs run on the matrix cores: v_mfma_f32_32x32x2_f32 (mixed) or
//    v_mfma_f64_16x16x4_f64 (FP64).  One workgroup per 32x32 output tile;
//    its four waves split the tile's K range, each streaming its A rows and
//    B columns through a wave-private LDS stage with coalesced loads, and
//    their partial tiles are added through LDS.  One launch covers every
//    (factor, body-column) tile of every shape.
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
// One workgroup computes one 32 x 32 output tile over a K range; its four
// waves take consecutive quarters of that range and add their partial tiles
// in LDS in wave order.  Each wave streams its quarter through its own LDS
// stage, one 128-byte run of K at a time (32 floats or 16 doubles):
//  * global -> registers, coalesced: lane l fetches the 16-byte piece l%8 of
//    the run of A row (and B column) l/8 + 8i, i < 4, so one load instruction
//    covers whole 128-byte lines of eight rows; the next run is fetched while
//    the current one is multiplied;
//  * registers -> LDS (rows padded by 16 bytes against bank conflicts), then
//    LDS -> MFMA fragments.  The stage belongs to one wave, whose LDS accesses
//    complete in order, so no workgroup barrier is needed inside the loop.
// The K index is permuted per lane inside a run (any bijection of K that A
// and B share leaves the product unchanged):
//  * f32, v_mfma_f32_32x32x2f32: lane l holds A[l%32][k] and B[k][l%32] for
//    k = 16 (l/32) + t, t < 16, one MFMA per t;
//  * f64, v_mfma_f64_16x16x4f64 (2 x 2 blocks of 16 x 16): lane l holds
//    A[l%16][k] and B[k][l%16] for k = 4 (l/16) + t, t < 4.
// A group's last column tile, when it holds at most GEMM_NARROW columns, is
// staged the same way but summed on the VALU (lane l: row l%32, columns
// l/32 + 2j), so the matrix cores do no work on padding columns there.
// Tiles are handed out XCD-aware: workgroup b runs on XCD b % 8 and takes
// tile (b % 8) * per_xcd + b / 8, so the column tiles of one (row tile, K
// range), which are consecutive in the tile list, run on one XCD and fetch
// their shared rows of A into its L2 once.  A K range is split over several
// tiles when there are few output tiles; split slices land in a partial
// buffer that a second kernel sums in a fixed order.  (Summing them in the
// kernel, by the slice that arrives last at a per-tile counter, needs an
// agent-scope release per workgroup: it measured 57 us against 15 + 5 us.)
// ---------------------------------------------------------------------------
constexpr int RUN_BYTES = 128;                      // one K run per LDS stage
constexpr int ROW_BYTES = RUN_BYTES + 16;           // padded LDS row
constexpr int STAGE_BYTES = 2 * 32 * ROW_BYTES;     // A and B runs of 32 rows / columns

template <class T>
struct __align__(16) Piece {  // 16 bytes of a run
    static constexpr int E = 16 / sizeof(T);
    T v[E];
};

// lane's piece of a run starting at k0 of one row (or column) p; zero past ke or when !ok
template <class T>
__device__ __forceinline__ Piece<T> load_piece(const T *__restrict__ p, int k, int ke, bool ok, bool vec) {
    constexpr int E = Piece<T>::E;
    Piece<T> r;
    if (ok && vec && k + E <= ke) {
        if constexpr (sizeof(T) == 4) {
            const float4 q = *reinterpret_cast<const float4 *>(p + k);
            r.v[0] = q.x; r.v[1] = q.y; r.v[2] = q.z; r.v[3] = q.w;
        } else {
            const double2 q = *reinterpret_cast<const double2 *>(p + k);
            r.v[0] = q.x; r.v[1] = q.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) r.v[e] = (ok && k + e < ke) ? p[k + e] : T(0);
    }
    return r;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class T>
__global__ __launch_bounds__(256) void gemm_kernel(int n_tiles, int per_xcd, const GemmTile *__restrict__ tiles,
                                                   const GemmGroup *__restrict__ groups, const T *__restrict__ Apool,
                                                   const T *__restrict__ B, const int64_t *__restrict__ b_col_off,
                                                   T *__restrict__ C, const int64_t *__restrict__ c_col_off,
                                                   T *__restrict__ partial, int64_t part_col_stride,
                                                   int64_t part_split_stride, int vec_ok) {
    constexpr int E = Piece<T>::E;                  // elements per 16-byte piece
    constexpr int KR = RUN_BYTES / sizeof(T);       // K per run: 32 floats or 16 doubles
    constexpr int LD = ROW_BYTES / sizeof(T);       // LDS row stride in elements
    __shared__ __align__(16) char smem[4][STAGE_BYTES];
    const int task = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (task >= n_tiles) return;  // uniform over the workgroup
    const GemmTile tl = tiles[task];
    const GemmGroup g = groups[tl.group];
    const T *A = Apool + g.a_off;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kq = (tl.k1 - tl.k0 + 4 * KR - 1) / (4 * KR) * KR;
    const int kb = min(tl.k1, tl.k0 + wave * kq), ke = min(tl.k1, kb + kq);
    const bool vec = vec_ok && (g.K % E) == 0;
    T *As = reinterpret_cast<T *>(smem[wave]);
    T *Bs = As + 32 * LD;

    // this lane's rows of A and columns of B for the global loads
    const int pc = lane & 7, pr = lane >> 3;
    const T *ap[4];
    const T *bp[4];
    bool aok[4], bok[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = tl.m0 + pr + 8 * i, c = tl.n0 + pr + 8 * i;
        aok[i] = r < g.M;
        bok[i] = c < g.ncol;
        ap[i] = A + (int64_t)(aok[i] ? r : 0) * g.K;
        bp[i] = B + b_col_off[g.col_begin + (bok[i] ? c : 0)];
    }
    Piece<T> ga[4], gb[4];
    auto fetch = [&](int k0) {
        if (vec && k0 + KR <= ke) {
            // the whole run lies inside K (a wave-uniform test): unconditional 16-byte loads;
            // rows and columns past the end read row / column 0 and are zeroed by stage(),
            // so nothing waits for these loads before the multiplications that follow
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ga[i] = *reinterpret_cast<const Piece<T> *>(ap[i] + k0 + E * pc);
                gb[i] = *reinterpret_cast<const Piece<T> *>(bp[i] + k0 + E * pc);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ga[i] = load_piece<T>(ap[i], k0 + E * pc, ke, aok[i], vec);
                gb[i] = load_piece<T>(bp[i], k0 + E * pc, ke, bok[i], vec);
            }
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            Piece<T> a = ga[i], b = gb[i];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                a.v[e] = aok[i] ? a.v[e] : T(0);
                b.v[e] = bok[i] ? b.v[e] : T(0);
            }
            *reinterpret_cast<Piece<T> *>(As + (pr + 8 * i) * LD + E * pc) = a;
            *reinterpret_cast<Piece<T> *>(Bs + (pr + 8 * i) * LD + E * pc) = b;
        }
    };

    // narrow tile: lane l sums row l%32 against columns l/32 + 2j, j < 4, of the staged run
    T nacc[4] = {T(0), T(0), T(0), T(0)};
    auto narrow_run = [&]() {
        const T *ar = As + (lane & 31) * LD;
#pragma unroll 1
        for (int kk = 0; kk < KR; kk += E) {
            const Piece<T> x = *reinterpret_cast<const Piece<T> *>(ar + kk);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const Piece<T> y = *reinterpret_cast<const Piece<T> *>(Bs + ((lane >> 5) + 2 * j) * LD + kk);
#pragma unroll
                for (int e = 0; e < E; ++e) nacc[j] += x.v[e] * y.v[e];
            }
        }
    };

    T val[16];
    const bool narrow = tl.narrow != 0;
    if (kb < ke) fetch(kb);
    if constexpr (sizeof(T) == 4) {
        const int c = lane & 31, h = lane >> 5;
        floatx16 acc = {};
        for (int k0 = kb; k0 < ke; k0 += KR) {
            stage();
            wave_lds_sync();
            if (k0 + KR < ke) fetch(k0 + KR);
            if (narrow) {
                narrow_run();
                wave_lds_sync();  // the next run's stores follow these reads
                continue;
            }
            float av[16], bv[16];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 x = *reinterpret_cast<const float4 *>(As + c * LD + 16 * h + 4 * j);
                const float4 y = *reinterpret_cast<const float4 *>(Bs + c * LD + 16 * h + 4 * j);
                av[4 * j] = x.x; av[4 * j + 1] = x.y; av[4 * j + 2] = x.z; av[4 * j + 3] = x.w;
                bv[4 * j] = y.x; bv[4 * j + 1] = y.y; bv[4 * j + 2] = y.z; bv[4 * j + 3] = y.w;
            }
            wave_lds_sync();  // the next run's stores follow these reads
#pragma unroll
            for (int t = 0; t < 16; ++t) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[t], bv[t], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) val[r] = acc[r];
    } else {
        const int q = lane >> 4, c16 = lane & 15;
        doublex4 acc[2][2] = {};
        for (int k0 = kb; k0 < ke; k0 += KR) {
            stage();
            wave_lds_sync();
            if (k0 + KR < ke) fetch(k0 + KR);
            if (narrow) {
                narrow_run();
                wave_lds_sync();
                continue;
            }
            double av[2][4], bv[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const double2 x = *reinterpret_cast<const double2 *>(As + (16 * u + c16) * LD + 4 * q + 2 * j);
                    const double2 y = *reinterpret_cast<const double2 *>(Bs + (16 * u + c16) * LD + 4 * q + 2 * j);
                    av[u][2 * j] = x.x; av[u][2 * j + 1] = x.y;
                    bv[u][2 * j] = y.x; bv[u][2 * j + 1] = y.y;
                }
            wave_lds_sync();
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int w = 0; w < 2; ++w)
                        acc[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][t], bv[w][t], acc[u][w], 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int w = 0; w < 2; ++w)
#pragma unroll
                for (int r = 0; r < 4; ++r) val[(2 * u + w) * 4 + r] = acc[u][w][r];
    }
    if (narrow)
#pragma unroll
        for (int r = 0; r < 16; ++r) val[r] = r < 4 ? nacc[r & 3] : T(0);
    // partial tiles of waves 1-3 through their own stages, added to wave 0's in wave order
    T *red = reinterpret_cast<T *>(smem[wave]);
    if (wave > 0)
#pragma unroll
        for (int r = 0; r < 16; ++r) red[r * 64 + lane] = val[r];
    __syncthreads();
    if (wave > 0) return;
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        const T *o = reinterpret_cast<const T *>(smem[w]);
#pragma unroll
        for (int r = 0; r < 16; ++r) val[r] += o[r * 64 + lane];
    }
    // output element of value slot r of this lane; false outside the group's matrix
    auto slot = [&](int r, int &row, int &col) -> bool {
        if (tl.narrow) {
            row = tl.m0 + (lane & 31);
            col = tl.n0 + (lane >> 5) + 2 * r;
            if (r >= 4) return false;
        } else if constexpr (sizeof(T) == 4) {
            // D layout (32x32x2): lane l, reg r -> row 8*(r/4) + 4*(l/32) + r%4, col l%32
            row = tl.m0 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
            col = tl.n0 + (lane & 31);
        } else {
            // D layout (16x16x4 f64, measured on gfx950): lane l, reg r -> row l/16 + 4 r, col l%16;
            // slot (2 u + w) * 4 + r holds block (u, w)
            const int bl = r / 4;
            row = tl.m0 + 16 * (bl >> 1) + (lane >> 4) + 4 * (r % 4);
            col = tl.n0 + 16 * (bl & 1) + (lane & 15);
        }
        return row < g.M && col < g.ncol;
    };
    if (!partial) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            int row, col;
            if (slot(r, row, col)) C[c_col_off[g.col_begin + col] + row] = val[r];
        }
        return;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        int row, col;
        if (slot(r, row, col))
            partial[tl.split * part_split_stride + (int64_t)(g.col_begin + col) * part_col_stride + row] = val[r];
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
// With n_slices > 1, lam is not read: the values are the sums of the split slices of
// the GEMM that produced them (in slice order, as gemm_reduce_kernel adds them).
template <class T>
__global__ __launch_bounds__(256) void project_kernel(BodyView bv, const T *__restrict__ lam, int rotate, int project,
                                                      double *__restrict__ out64, void *__restrict__ srcS,
                                                      void *__restrict__ srcL, int src_prec,
                                                      const T *__restrict__ part, int n_slices, int64_t split_stride,
                                                      int64_t col_stride, const int32_t *__restrict__ col_of_body) {
    __shared__ double sh[4][6];
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    const T *pb = n_slices > 1 ? part + (int64_t)col_of_body[b] * col_stride : nullptr;
    auto val = [&](int64_t j) -> double {
        if (n_slices <= 1) return (double)lam[off + j];
        T s = T(0);
        for (int sp = 0; sp < n_slices; ++sp) s += pb[sp * split_stride + j];
        return (double)s;
    };
    // the projection reads every value twice; the first pass keeps them here (each
    // thread reads back only its own entries)
    constexpr int CACHE = 2048;
    __shared__ double cache[CACHE];
    const bool cached = project && (kind == MFS_LAPLACE ? n : 3 * n) <= CACHE;
    if (kind == MFS_LAPLACE) {
        double s[1] = {0.0};
        if (project) {
            for (int j = threadIdx.x; j < n; j += blockDim.x) {
                const double v = val(j);
                if (cached) cache[j] = v;
                s[0] += v;
            }
            block_sum<1>(s, reinterpret_cast<double(*)[1]>(sh));
        }
        const double mean = project ? s[0] / n : 0.0;
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            const double v = (cached ? cache[j] : val(j)) - mean;
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
            double v[3] = {val(3 * j), val(3 * j + 1), val(3 * j + 2)};
            if (cached) {
                cache[3 * j] = v[0];
                cache[3 * j + 1] = v[1];
                cache[3 * j + 2] = v[2];
            }
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
        double v[3];
        if (cached) {
            v[0] = cache[3 * j];
            v[1] = cache[3 * j + 1];
            v[2] = cache[3 * j + 2];
        } else {
            v[0] = val(3 * j);
            v[1] = val(3 * j + 1);
            v[2] = val(3 * j + 2);
        }
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

// dJ/d(net) from t = dJ/ds_0 (lambda layout; the completion strengths enter b
// = -S s_0 with the self block): Laplace s_0 = (q/N) 1 gives dJ/dq = mean(t);
// Stokes s_0 = K_N G^{-1} [f; t] gives dJ/d[f; t] = G^{-1} K_N^T t (G symmetric).
__global__ __launch_bounds__(256) void grad_net_kernel(BodyView bv, const double *__restrict__ t,
                                                       double *__restrict__ gnet) {
    __shared__ double sh[4][6];
    const int64_t b = blockIdx.x;
    const int kind = bv.kind[b];
    const int n = bv.n_src[b];
    const int64_t off = bv.lam_off[b];
    const int64_t row0 = bv.src_row[b];
    if (kind == MFS_LAPLACE) {
        double s[1] = {0.0};
        for (int j = threadIdx.x; j < n; j += blockDim.x) s[0] += t[off + j];
        block_sum<1>(s, reinterpret_cast<double(*)[1]>(sh));
        if (threadIdx.x == 0) gnet[bv.net_off[b]] = s[0] / n;
        return;
    }
    double w[6] = {0, 0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const double *v = t + off + 3 * j;
        const double *d = bv.src_off64 + 4 * (row0 + j);
        double c[3];
        cross3(d, v, c);
        w[0] += v[0]; w[1] += v[1]; w[2] += v[2];
        w[3] += c[0]; w[4] += c[1]; w[5] += c[2];
    }
    block_sum<6>(w, sh);
    if (threadIdx.x == 0) {
        const double *Gi = bv.gram_inv + 36 * b;
        for (int r = 0; r < 6; ++r) {
            double acc = 0.0;
            for (int c = 0; c < 6; ++c) acc += Gi[6 * r + c] * w[c];
            gnet[bv.net_off[b] + r] = acc;
        }
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
                    const int64_t *c_col_off, float *partial, hipStream_t s, bool sum_slices) {
    if (G.n_tiles == 0) return MFS_OK;
    float *part = G.n_split > 1 ? partial : nullptr;
    const int per_xcd = (G.n_tiles + 7) / 8;
    gemm_kernel<float><<<8 * per_xcd, 256, 0, s>>>(G.n_tiles, per_xcd, G.tiles, G.groups, Apool, B, b_col_off, C,
                                                          c_col_off, part, G.part_col_stride, G.part_split_stride, G.vec4);
    MFS_HIP_TRY(hipGetLastError());
    if (part && sum_slices) {
        gemm_reduce_kernel<float><<<dim3(G.n_cols, (unsigned)((G.part_col_stride + 255) / 256)), 256, 0, s>>>(
            G.col_group, G.groups, part, G.part_col_stride, G.part_split_stride, G.n_split, C, c_col_off);
        MFS_HIP_TRY(hipGetLastError());
    }
    return MFS_OK;
}

int launch_gemm_f64(const GemmLaunch &G, const double *Apool, const double *B, const int64_t *b_col_off, double *C,
                    const int64_t *c_col_off, double *partial, hipStream_t s, bool sum_slices) {
    if (G.n_tiles == 0) return MFS_OK;
    double *part = G.n_split > 1 ? partial : nullptr;
    const int per_xcd = (G.n_tiles + 7) / 8;
    gemm_kernel<double><<<8 * per_xcd, 256, 0, s>>>(G.n_tiles, per_xcd, G.tiles, G.groups, Apool, B, b_col_off, C,
                                                            c_col_off, part, G.part_col_stride, G.part_split_stride, G.vec4);
    MFS_HIP_TRY(hipGetLastError());
    if (part && sum_slices) {
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

template <class S, class D>
__global__ void cast_kernel(int64_t n, const S *__restrict__ in, D *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (D)in[i];
}

int launch_cast(int64_t n, const void *in, bool in_f32, void *out, hipStream_t s) {
    if (n <= 0) return MFS_OK;
    const unsigned grid = (unsigned)((n + 255) / 256);
    if (in_f32) cast_kernel<float, double><<<grid, 256, 0, s>>>(n, (const float *)in, (double *)out);
    else cast_kernel<double, float><<<grid, 256, 0, s>>>(n, (const double *)in, (float *)out);
    MFS_HIP_TRY(hipGetLastError());
    return MFS_OK;
}

int launch_project(const BodyView &bv, const void *lam, bool lam_f32, bool rotate, bool project, double *out64,
                   void *srcS, void *srcL, int src_prec, hipStream_t s, const SplitSlices *slices) {
    if (bv.n_body == 0) return MFS_OK;
    const SplitSlices none;
    const SplitSlices &sl = slices && slices->n > 1 ? *slices : none;
    if (lam_f32)
        project_kernel<float><<<(unsigned)bv.n_body, 256, 0, s>>>(
            bv, (const float *)lam, rotate, project, out64, srcS, srcL, src_prec, (const float *)sl.part, sl.n,
            sl.split_stride, sl.col_stride, sl.col_of_body);
    else
        project_kernel<double><<<(unsigned)bv.n_body, 256, 0, s>>>(
            bv, (const double *)lam, rotate, project, out64, srcS, srcL, src_prec, (const double *)sl.part, sl.n,
            sl.split_stride, sl.col_stride, sl.col_of_body);
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

int launch_grad_net(const BodyView &bv, const double *t, double *gnet, hipStream_t s) {
    if (bv.n_body == 0) return MFS_OK;
    grad_net_kernel<<<(unsigned)bv.n_body, 256, 0, s>>>(bv, t, gnet);
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
