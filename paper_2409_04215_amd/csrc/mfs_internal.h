// Internal declarations shared by the libmfs translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mfs.h"

namespace mfs {

// ---------------------------------------------------------------------------
// Error state
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

#define MFS_HIP_TRY(expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::mfs::fail(MFS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MFS_TRY(expr)          \
    do {                       \
        int s_ = (expr);       \
        if (s_ < 0) return s_; \
    } while (0)

constexpr double PI = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Device buffer (library-owned memory)
// ---------------------------------------------------------------------------
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            ptr = o.ptr;
            bytes = o.bytes;
            o.ptr = nullptr;
            o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    int reserve(size_t n);                 // grows (contents not kept)
    int upload(const void *host, size_t n, hipStream_t s);
    template <class T> T *as() const { return reinterpret_cast<T *>(ptr); }
};

// ---------------------------------------------------------------------------
// Pair-sum operands.
//
// Coordinates are split as world = centre (FP64, per body) + offset, where the
// offset (world axes, relative to the body centre) is small.  The mixed kernels
// keep offsets and strengths in FP32 and form d = (float(c_t - c_s) + xt) - ys,
// which keeps the FP32 rounding of d relative to |d| rather than to the
// distance from the origin.
// ---------------------------------------------------------------------------
struct SrcS32 { float4 pos; float4 str; };   // Stokes mixed: offset, strength (w unused)
struct SrcS64 { double pos[4]; double str[4]; };
typedef float4 SrcL32;                         // Laplace mixed: offset xyz, strength w
struct SrcL64 { double v[4]; };

// One unit of pair-sum work: targets [t0, t1) of one system against the
// sources of bodies [b0, b1) of the same system; results go to split slice
// `split` at output offset out0 (+ dim per target).
struct P2PItem {
    int64_t out0;
    double scale;        // 1/(4 pi) or 1/(8 pi mu)
    int32_t t0, t1;
    int32_t b0, b1;
    int32_t sys;
    int32_t split;
    int32_t kind;
    int32_t pad;
};

// Everything one pair-sum launch reads and writes (device pointers).
struct P2PLaunch {
    int prec = MFS_MIXED;
    bool skip_same = true;
    bool accumulate = false;
    double alpha = 1.0;              // extra factor on the pair sum (e.g. -1 for b = -u0)
    const double *centre = nullptr;  // [n_body][3] FP64 body centres
    const int32_t *trg_body = nullptr;
    const int32_t *src_ptr = nullptr;     // [n_body+1] source rows per body
    const int32_t *sys_active = nullptr;  // [n_sys] or null
    const void *trg_off = nullptr;        // float4 / double4 [n_trg] offsets from the body centre
    const void *srcS = nullptr;           // SrcS32 / SrcS64 [n_src] (Stokes bodies)
    const void *srcL = nullptr;           // SrcL32 / SrcL64 [n_src] (Laplace bodies)
    double *out = nullptr;                // final output [n_val]
    double *partial = nullptr;            // [n_split][n_val] when n_split > 1
    const double *addend = nullptr;       // added once to the output (may be null)
    int64_t n_val = 0;                    // output length
    hipEvent_t ev_start = nullptr;        // optional events recorded right around the pair kernel
    hipEvent_t ev_stop = nullptr;
};

// Host-side description of a pair-sum launch.
struct P2PPlan {
    std::vector<P2PItem> items;
    int n_split = 1;
    int tpl = 1;
    bool persistent = false;     // fixed grid + work-queue counter instead of one workgroup per item
    int persistent_grid = 2048;  // workgroups of a persistent launch
    DevBuf d_items;
    DevBuf d_counter;            // int work-queue counter (persistent mode)
};

// items for targets grouped by body (body_trg_ptr), bodies grouped by system;
// out_ptr[b] = output offset of body b's first target; dim_of_body 1 or 3.
int build_p2p_items(P2PPlan &pp, int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                    const int64_t *body_src_ptr, const int64_t *out_ptr, const int32_t *kind_of_body,
                    double mu, int tpl, int min_items, hipStream_t s);

// The same items written into caller-provided host arrays, with no heap
// allocation: out_ptr may be null (then out_dim * body_trg_ptr[b]) and
// kind_of_body null (then every body has `kind`).  items, work and order need
// room for cap entries; on return items[0..*n_items) are in launch order.
// MFS_EINVAL when more than cap items would be needed.
int generate_p2p_items(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                       const int64_t *body_src_ptr, const int64_t *out_ptr, int out_dim,
                       const int32_t *kind_of_body, int kind, double mu, int tpl, int min_items, P2PItem *items,
                       double *work, int32_t *order, P2PItem *sorted, int64_t cap, int64_t *n_items, int *n_split);

// A pair-sum launch's items wherever they live (device pointers).
struct P2PItems {
    const P2PItem *items = nullptr;
    int n_items = 0;
    int n_split = 1;
    int tpl = 1;
    bool persistent = false;
    int persistent_grid = 2048;
    int *counter = nullptr;  // persistent mode only
};
P2PItems items_of(const P2PPlan &pp);

// kernels (p2p_kernels.hip)
int launch_p2p(const P2PItems &it, const P2PLaunch &L, hipStream_t s);
inline int launch_p2p(const P2PPlan &pp, const P2PLaunch &L, hipStream_t s) { return launch_p2p(items_of(pp), L, s); }

// Standalone conversion: FP64 world points to the split representation.
int launch_body_refpoint(int64_t n_body, const int32_t *src_ptr, const int32_t *trg_ptr, const double *src_xyz,
                         const double *trg_xyz, double *centre, hipStream_t s);
int launch_make_trg_off(int64_t n_trg, const double *xyz, const int32_t *trg_body, const double *centre,
                        int prec, void *out, hipStream_t s);
int launch_make_src(int64_t n_src, int kind, const double *xyz, const int32_t *src_body, const double *centre,
                    const double *str, int prec, void *out, hipStream_t s);
int launch_fill_body_ids(int64_t n_body, const int32_t *ptr, int32_t *ids, hipStream_t s);

// Position gradients of the pair sums (p2p_backward.hip): lane vectors indexed like the
// forward output, gradient [n_lane][3].
int launch_p2p_grad(const P2PPlan &pp, const P2PLaunch &L, const double *lane_vec, int64_t n_lane, hipStream_t s);

// Derived fields of the representation (field_kernels.hip): items of one target
// per lane; L.srcS (pressure, traction) or L.srcL (Laplace gradient) hold the
// sources; out [n_trg] (pressure) or [n_trg][3]; normal [n_trg][3] (traction).
enum { MFS_FIELD_PRESSURE = 0, MFS_FIELD_TRACTION = 1, MFS_FIELD_LAPLACE_GRADIENT = 2 };
int launch_field(int field, const P2PPlan &pp, const P2PLaunch &L, const double *normal, int64_t n_trg,
                 hipStream_t s);
// eps[i] = |u_i - g_i| / |g_i| with g the rigid motion (or potential) of body[i] at offset off64[i]
int launch_residual(int64_t n, const int32_t *body, const int32_t *kind, const int64_t *net_off, const double *off64,
                    const double *u, const int64_t *u_off, const double *motion, double *eps, hipStream_t s);

// ---------------------------------------------------------------------------
// Block (one-body) kernels (block_kernels.hip)
// ---------------------------------------------------------------------------
// One workgroup's task: output tile (m0, n0) of a group over K range [k0, k1), split slice
// `split`; `narrow`: the tile has at most GEMM_NARROW columns and is summed on the VALU
// instead of the matrix cores.
struct GemmTile { int32_t group, m0, n0, k0, k1, split, narrow; };
constexpr int GEMM_NARROW = 8;
struct GemmGroup {
    int32_t M, K;             // A is M x K row-major (lda = K)
    int32_t col_begin, ncol;  // columns [col_begin, col_begin+ncol) of the column table
    int64_t a_off;            // element offset of A in the factor pool
};
// One grouped-GEMM launch (device tables built at plan creation).
struct GemmLaunch {
    int n_tiles = 0;
    int n_split = 1;
    int n_cols = 0;
    const GemmTile *tiles = nullptr;
    const GemmGroup *groups = nullptr;
    const int32_t *col_group = nullptr;  // [n_cols] group of every column
    int64_t part_col_stride = 0;         // partial buffer: [n_split][n_cols][part_col_stride]
    int64_t part_split_stride = 0;
    int vec4 = 0;  // every A row start and B column start is 16-byte aligned (float4 / double2 loads)
};

// sum_slices = false leaves a split GEMM's slices in `partial` (C is not written): the
// consumer adds them (SplitSlices).
int launch_gemm_f32(const GemmLaunch &G, const float *Apool, const float *B, const int64_t *b_col_off, float *C,
                    const int64_t *c_col_off, float *partial, hipStream_t s,
                    bool sum_slices = true);
int launch_gemm_f64(const GemmLaunch &G, const double *Apool, const double *B, const int64_t *b_col_off, double *C,
                    const int64_t *c_col_off, double *partial, hipStream_t s,
                    bool sum_slices = true);

// Per-body view used by rotation / projection / extraction kernels.
struct BodyView {
    int64_t n_body;
    const int32_t *kind;       // [n_body]
    const int32_t *n_src;      // [n_body]
    const int32_t *n_trg;
    const int64_t *gam_off;    // [n_body] offset in gamma layout
    const int64_t *lam_off;    // [n_body] offset in lambda layout
    const int64_t *net_off;    // [n_body] offset in net layout
    const int32_t *src_row;    // [n_body] first source row (point index)
    const int32_t *trg_row;
    const double *rot;         // [n_body][9]
    const double *gram_inv;    // [n_body][36] (Stokes bodies)
    const double *src_off64;   // [n_src][4] world-axis offsets of the proxies
    const double *trg_off64;   // [n_trg][4] world-axis offsets of the collocation points
    int dirichlet;             // 1: capacitance / resistance formulation (no projection)
};

// in (world frame fp64) -> out (shape frame, float or double); gamma layout (M points per body)
// or lambda layout (N points per body)
int launch_rotate_in(const BodyView &bv, const double *in, void *out, bool out_f32, bool lam_layout, hipStream_t s);
// shape frame (float or double) -> world frame fp64
int launch_rotate_out(const BodyView &bv, const void *in, bool in_f32, double *out, bool lam_layout, hipStream_t s);
// out[i] = in[i] converted float -> double (in_f32) or double -> float, i < n
int launch_cast(int64_t n, const void *in, bool in_f32, void *out, hipStream_t s);
// lam (lambda layout) -> optionally rotated to the world frame, optionally (I - L); written to out64
// (may alias lam when lam is fp64 and rotate is false) and/or into the pair-sum source records
// srcS / srcL (chosen by body kind; either may be null) of precision src_prec
// Split-K slices of a GEMM whose columns are bodies, read in place of its output:
// value j of body b = sum over sp < n of part[sp * split_stride + col_of_body[b] * col_stride + j],
// added in slice order as the GEMM's own reduction does.
struct SplitSlices {
    const void *part = nullptr;
    int n = 1;
    int64_t split_stride = 0, col_stride = 0;
    const int32_t *col_of_body = nullptr;
};
int launch_project(const BodyView &bv, const void *lam, bool lam_f32, bool rotate, bool project, double *out64,
                   void *srcS, void *srcL, int src_prec, hipStream_t s, const SplitSlices *slices = nullptr);
int launch_completion(const BodyView &bv, const double *net, double *s0, void *srcS, void *srcL, int src_prec,
                      hipStream_t s);
int launch_extract(const BodyView &bv, const double *lam, const double *s0, double *out, double *sigma,
                   hipStream_t s);
// Dirichlet data at the collocation points: phi 1_M or v + omega x (x - c) (gamma layout)
int launch_dirichlet_rhs(const BodyView &bv, const double *data, double *b, hipStream_t s);
int launch_grad_lambda(const BodyView &bv, const double *grad_out, double *glam, hipStream_t s);
int launch_grad_net(const BodyView &bv, const double *t, double *gnet, hipStream_t s);
int launch_set_src_strength(const BodyView &bv, const double *str, void *srcS, void *srcL, int prec, hipStream_t s);
int launch_body_grad_reduce(int64_t n_body, const int32_t *trg_ptr, const int32_t *src_ptr, const double *gt,
                            const double *gs, double *grad_c, hipStream_t s);
int launch_make_factor(int rows, int cols, const double *src, int64_t ld, bool transposed, const double *rs,
                       const double *cs, double *d64, float *d32, hipStream_t s);

// setup
// S_L (column-major M x N blocks of dim) or, with plain, the bare block S^(kk)
int launch_assemble_SL(int kind, int M, int N, const double *trg, const double *src, const double *gram_inv6,
                       double mu, bool plain, double *SL, double *work, hipStream_t s);
int launch_scale_rows_to_f32(int rows, int cols, const double *src, int64_t ld_src, const double *row_scale,
                             const double *col_scale, double *dst64, float *dst32, hipStream_t s);

// ---------------------------------------------------------------------------
// Krylov vector kernels (krylov_kernels.hip)
// ---------------------------------------------------------------------------
struct VecChunk { int64_t begin, end; int32_t sys; int32_t pad; };
int launch_multi_dot(int n_chunk, const VecChunk *chunks, const double *V, int64_t ldv, int nvec, const double *w,
                     double *partial, int ld_partial, hipStream_t s);
int launch_reduce_sys(int n_sys, const int32_t *sys_chunk_ptr, const double *partial, int ld_partial, int nval,
                      double *out, int ld_out, hipStream_t s);
int launch_multi_axpy(int n_chunk, const VecChunk *chunks, const double *V, int64_t ldv, int nvec,
                      const double *coef, int ld_coef, double sign, double *w, hipStream_t s);
int launch_scale_sys(int n_chunk, const VecChunk *chunks, const double *w, const double *scale, int ld_scale,
                     double *out, hipStream_t s);
// w += sign * V coef (as launch_multi_axpy), then partial[c][i] = D[i] . w over chunk c for i < ndot
// (as launch_multi_dot on the updated w), in one kernel with the same arithmetic order.
int launch_axpy_dot(int n_chunk, const VecChunk *chunks, const double *V, int64_t ldv, int nvec, const double *coef,
                    int ld_coef, double sign, double *w, const double *D, int64_t ldd, int ndot, double *partial,
                    int ld_partial, hipStream_t s);
int launch_sub(int64_t n, const double *a, const double *b, double *out, hipStream_t s);
int launch_add_inplace(int64_t n, const double *a, double *out, hipStream_t s);
int launch_fill(int64_t n, double v, double *out, hipStream_t s);
int launch_check_finite(int64_t n, const double *x, int32_t *flag, hipStream_t s);

// Device state of the GMRES least-squares problems, one per system: the Hessenberg
// columns are reduced by Givens rotations as they arrive, so |g_{j+1}| is the
// residual estimate of iteration j (Saad & Schultz).  Arrays are per system, with
// the leading dimensions given; R holds the rotated columns packed (column j at
// j(j+1)/2, rows 0..j).
struct GivensState {
    int n_sys = 0, cap = 0, ldh = 0;   // systems, largest Krylov dimension, CGS row stride
    const double *dots = nullptr;      // [n_sys][2][ldh] CGS coefficients of both passes
    const double *nrm2 = nullptr;      // [n_sys] squared norm of the orthogonalised vector
    const double *target = nullptr;    // [n_sys] absolute residual target
    const double *beta = nullptr;      // [n_sys] initial residual norm
    double *R = nullptr;               // [n_sys][cap (cap + 1) / 2]
    double *cs = nullptr, *sn = nullptr;  // [n_sys][cap]
    double *g = nullptr;               // [n_sys][cap + 1]
    int32_t *k = nullptr;              // [n_sys] columns of the least-squares problem
    int32_t *live = nullptr;           // [n_sys] systems still iterating (the matvec's mask)
    double *scale = nullptr;           // [n_sys] 1 / h_{j+1,j} for live systems, else 0
    double *est = nullptr;             // [n_sys] residual estimate
};
// Status block of one iteration, written by the step kernel into host-mapped memory:
// est[n_sys] (residual estimates), then flag[n_sys] (bit 0: live, bit 1: non-finite column).
int launch_givens_init(const GivensState &st, hipStream_t s);

// Batched FP64 Householder QR of column-major m x n matrices A (leading dimension m, m >= n,
// n <= 8192), factor_kernels.hip, blocked in panels of 32 columns (compact WY, trailing
// updates and the accumulation of Q on the FP64 matrix cores): A is overwritten by R (upper
// triangle) and the reflectors, Q (m x n, leading dimension m) and X = R^-1 (n x n, leading
// dimension n) are written, and ratio[b] = 1 / (||R||_F ||R^-1||_F).  scratch: device
// memory of qr_scratch_doubles(batch, n) doubles (tau, column norms and the panels' T factors).
size_t qr_scratch_doubles(int batch, int n);
int qr_inverse_batched(int batch, double *A, int m, int n, int64_t stride_a, double *Q, int64_t stride_q, double *X,
                       int64_t stride_x, double *scratch, double *ratio, hipStream_t s);
// Iteration j's last reduction (|w|^2 per system from the chunk partials, into nrm2, which
// must be st.nrm2) and its Givens step, writing the iteration's status block.
int launch_givens_step(const GivensState &st, const int32_t *sys_chunk_ptr, const double *partial, int ld_partial,
                       double *nrm2, int j, double *status_est, int32_t *status_flag, hipStream_t s);
int launch_givens_solve(const GivensState &st, double *coef, int ld_coef, int nvec, hipStream_t s);

}  // namespace mfs
