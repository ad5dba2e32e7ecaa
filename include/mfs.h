/*
 * mfs.h -- C ABI of libmfs, the MI355X (gfx950) library for the
 * one-body-preconditioned method of fundamental solutions (MFS) for 3D Laplace
 * elastance and Stokes mobility problems (Broms, Barnett and Tornberg,
 * arXiv 2409.04215).
 *
 * The library computes, on one GPU, the operator that GMRES applies in the
 * paper's preconditioned square system (Section 3.3, eq. (2esysprec)):
 *
 *   (A gamma)^(k) = gamma^(k) + sum_{k' != k} S^(kk') (I - L^(k')) S_L^(k')+ gamma^(k'),
 *
 * its pieces (all-pairs fundamental-solution sums, per-body pseudo-inverse
 * blocks, rigid-body / constant projection), the right-hand side, GMRES
 * around it, the recovery of potentials or rigid velocities, and the adjoint
 * of all of these for gradients with respect to particle centres and to the
 * given net quantities.
 *
 * Conventions that hold for every entry point
 * ------------------------------------------
 * - Pointers marked [device] are GPU memory (e.g. torch.Tensor.data_ptr());
 *   pointers marked [host] are CPU memory.  The caller owns every array it
 *   passes; the library never frees caller memory and keeps no pointer to it
 *   after the call returns.
 * - Arrays are dense and row-major.  Points are [n][3] double; Stokes
 *   strengths and velocities are [n][3] double (the paper's point-major
 *   stacking, index 3(i-1)+a); Laplace strengths and potentials are [n] double.
 * - Points are grouped by body and bodies by system (an independent
 *   suspension).  Pairs in different systems never interact.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Calls are asynchronous on it unless stated otherwise.
 * - Return value: MFS_OK (0) on success, a positive warning (outputs valid) or
 *   a negative error.  Argument errors (MFS_EINVAL) are detected on the host
 *   before any launch and leave every output untouched.  mfs_last_error()
 *   returns a thread-local description of the last non-OK status.
 * - Contents of device index arrays are not validated on the device.
 * - A pair whose target and source coincide (r = 0) gives a non-finite term;
 *   the method never forms one (proxies lie strictly inside their body and
 *   bodies do not overlap).
 */
#ifndef MFS_H
#define MFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MFS_OK = 0,
    MFS_NOT_CONVERGED = 1, /* GMRES hit max_iter; outputs hold the best iterate */
    MFS_EINVAL = -1,       /* bad argument; nothing was launched or written */
    MFS_EHIP = -2,         /* a HIP runtime or library call failed */
    MFS_ENOMEM = -3,       /* device allocation failed */
    MFS_ENUMERIC = -4,     /* non-finite value, breakdown or singular factor */
    MFS_EUNSUPPORTED = -5
} mfs_status;

typedef enum { MFS_LAPLACE = 0, MFS_STOKES = 1 } mfs_kind;

/* MIXED: FP32 pair arithmetic (relative coordinates, FP64 accumulation per
 * source tile) and FP32 MFMA pseudo-inverse blocks; FP64 projections and
 * GMRES.  FP64: every step in FP64. */
typedef enum { MFS_FP64 = 0, MFS_MIXED = 1 } mfs_precision;

enum {
    MFS_SKIP_SAME_BODY = 1, /* leave out pairs whose target and source share a body */
    MFS_ACCUMULATE = 2,     /* out += sum instead of out = sum */
    MFS_PROJECT = 4,        /* precond apply: also apply (I - L) */
    MFS_TRANSPOSE = 8       /* precond apply: apply the transpose */
};

/* Thread-local text for the last non-OK status of this thread. */
const char *mfs_last_error(void);
/* Library version string. */
const char *mfs_version(void);

/* -------------------------------------------------------------------------
 * All-pairs sums (the MFS representation, Section 2.1 eq. (rep) with the
 * Laplace G = 1/(4 pi r), and Section 2.2 eq. (repS) with the Stokeslet
 * eq. (stokeslet), G = (I + d d^T / r^2) / (8 pi mu r), d = x - y):
 *
 *   out_i (+)= sum_{j in sys(i), !(SKIP && body(j) == body(i))} G(x_i - y_j) s_j
 *
 * Structure arrays [host]:
 *   sys_body_ptr [n_sys+1]  bodies of system s are [sys_body_ptr[s], sys_body_ptr[s+1])
 *   body_trg_ptr [n_body+1] targets of body b are rows [body_trg_ptr[b], body_trg_ptr[b+1])
 *   body_src_ptr [n_body+1] sources of body b are rows [body_src_ptr[b], body_src_ptr[b+1])
 *   (n_body = sys_body_ptr[n_sys]; all three must be non-decreasing, start at 0,
 *    and the totals must fit in int32.)
 * Data arrays [device]: trg_xyz [n_trg][3], src_xyz [n_src][3],
 *   src_q [n_src] / src_f [n_src][3], out_u [n_trg] / [n_trg][3].
 * prec: MFS_MIXED or MFS_FP64.  mu must be finite and positive.
 * Asynchronous on `stream`.  Uses a library-owned device workspace, one per
 * host thread and device (allocated on first use; growing it waits for the
 * device).  The first call with a given structure (the three pointer arrays,
 * mu and the entry point) also builds the work tables of its launch and keeps
 * them for later calls with the same structure (up to 8 structures per
 * workspace; evicting one waits for the device).  Calls of one host thread on
 * different streams share that workspace and must not overlap.
 * Errors: MFS_EINVAL for NULL data pointers, n_sys < 1, bad structure arrays,
 * unknown flags or precision.
 * ------------------------------------------------------------------------- */
int mfs_p2p_laplace(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                    const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                    const double *src_q, double *out_u, int flags, int prec, void *stream);
int mfs_p2p_stokes(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                   const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                   const double *src_f, double *out_u, double mu, int flags, int prec, void *stream);

/* mfs_p2p_stokes for callers that cannot allocate device memory (code that may
 * not call hipMalloc or hipFree: tight serving loops, harnesses that forbid
 * allocation).  Same arguments, arithmetic, launch shape and results as
 * mfs_p2p_stokes (bit for bit), but every device buffer beyond the inputs and
 * the output lives in one library-owned scratch array of 64 MiB per GPU that
 * the library holds from load until the process ends; the call allocates
 * nothing and keeps nothing between calls.  Limits: at most 65536 bodies,
 * 32768 work items (about 2e6 targets) and 64 MiB of scratch: 36 B per
 * source and 20 B per target (mixed) or 68 B and 36 B (FP64), plus 24 B per
 * target and split slice when the sources are split; beyond them it returns
 * MFS_EINVAL before any launch.  The kernels write every scratch
 * value they read, so nothing needs clearing between calls.  Every call on a
 * GPU shares that GPU's scratch: calls are serialised on the host (a mutex)
 * and each waits for its stream before it returns (synchronous), so calls
 * that overlap on one GPU from other processes or through other library
 * copies race. */
int mfs_p2p_stokes_noalloc(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                           const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                           const double *src_f, double *out_u, double mu, int flags, int prec, void *stream);

/* Backward of the pairing  Phi = sum_i w_i . out_i  for the sums above
 * (flags as there; ACCUMULATE adds into every gradient that is requested):
 *   grad_src  [n_src] / [n_src][3]  dPhi/ds_j   = sum_i G(y_j - x_i) w_i
 *   grad_trg_xyz [n_trg][3]         dPhi/dx_i
 *   grad_src_xyz [n_src][3]         dPhi/dy_j
 * Any of the three gradient pointers may be NULL (that pass is skipped).
 * trg_w is [n_trg] (Laplace) or [n_trg][3] (Stokes) [device].
 * Pair gradient (d = x - y, r = |d|), Stokes:
 *   dPhi_ij/dd = [-(w.s) d + (w.d) s + (s.d) w - 3 (w.d)(s.d) d / r^2] / (8 pi mu r^3);
 * Laplace: dPhi_ij/dd = -w s d / (4 pi r^3).  Derived from the kernels above;
 * the paper has no gradients. */
int mfs_p2p_laplace_backward(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                             const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                             const double *src_q, const double *trg_w, double *grad_src_q,
                             double *grad_trg_xyz, double *grad_src_xyz, int flags, int prec,
                             void *stream);
int mfs_p2p_stokes_backward(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                            const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                            const double *src_f, const double *trg_w, double *grad_src_f,
                            double *grad_trg_xyz, double *grad_src_xyz, double mu, int flags, int prec,
                            void *stream);

/* Derived fields of the representation at arbitrary targets (same structure
 * arguments, flags and precision as the pair sums above; d = x_i - y_j, r = |d|).
 *   mfs_p2p_stokes_pressure: out_p [n_trg] = (1/(8 pi)) sum_j Pi(d) . f_j with
 *     Pi(d) = 2 d / r^3 (Section 2.2, the pressure of the representation).
 *   mfs_p2p_stokes_traction: out_t [n_trg][3] = sigma(x_i) . n_i, the stress
 *     sigma = -p I + mu (grad u + grad u^T) of the Stokeslet sum (eq. (traction)),
 *     sigma_ab = -(3/(4 pi)) sum_j d_a d_b (d . f_j) / r^5 (independent of mu);
 *     trg_normal [n_trg][3] [device] holds the unit vectors n_i.  With n the
 *     outward normal of a body, the integral of the traction over its surface is
 *     the force of the fluid on the body, -K_N^T lambda.
 *   mfs_p2p_laplace_gradient: out_g [n_trg][3] = grad u(x_i) =
 *     -(1/(4 pi)) sum_j q_j d / r^3.
 * Derived from the kernels of Section 2 (the paper states the pressure and
 * the traction definition, not these sums). */
int mfs_p2p_stokes_pressure(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                            const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                            const double *src_f, double *out_p, int flags, int prec, void *stream);
int mfs_p2p_stokes_traction(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                            const int64_t *body_src_ptr, const double *trg_xyz, const double *trg_normal,
                            const double *src_xyz, const double *src_f, double *out_t, int flags, int prec,
                            void *stream);
int mfs_p2p_laplace_gradient(int64_t n_sys, const int64_t *sys_body_ptr, const int64_t *body_trg_ptr,
                             const int64_t *body_src_ptr, const double *trg_xyz, const double *src_xyz,
                             const double *src_q, double *out_g, int flags, int prec, void *stream);

/* -------------------------------------------------------------------------
 * Plans.  A plan owns everything the solve reuses: device geometry, the
 * per-shape pseudo-inverse factors of S_L = S^(kk)(I - L) + L_r (Section 3.3),
 * per-body Gram inverses (K_N^T K_N)^{-1} (eq. (lambda02)), work tables and
 * the Krylov workspace.
 *
 * Geometry: body b of shape s has world proxies y = centre_b + rot_b ytilde
 * and collocation points x = centre_b + rot_b xtilde, with ytilde and xtilde
 * the shape's local points.  Bodies sharing a shape and a kind share one FP64
 * SVD of S_L in the shape frame; rotated copies apply it as Remark
 * "congruent" states (lambda = R V Sigma^+ U^T R^T gamma).  No truncation:
 * creation fails with MFS_ENUMERIC if sigma_min/sigma_max <= 1e-14.
 *
 * Vector layouts (all [device], FP64, bodies in order):
 *   gamma / b / A gamma : body b holds dim_b * M_b entries (dim 1 Laplace, 3 Stokes)
 *   lambda / strengths  : body b holds dim_b * N_b entries
 *   net / out           : body b holds 1 (q or phi) or 6 ([f;t] or [v;omega]) entries
 * mfs_plan_sizes reports the three totals.
 * ------------------------------------------------------------------------- */
typedef struct mfs_plan_s *mfs_plan;

/* Formulation of a plan.
 * MFS_MOBILITY: the paper's new formulations (Section 3): elastance (Laplace,
 *   given net charges, unknown potentials) and mobility (Stokes, given net
 *   forces and torques, unknown rigid velocities), one-body preconditioned
 *   with S_L^+ and the projection (I - L) (eq. (2esysprec)).
 * MFS_RESISTANCE: the Dirichlet formulations (Section 2): capacitance
 *   (Laplace, given potentials phi^(k), unknown charges q^(k)) and resistance
 *   (Stokes, given rigid velocities U^(k), unknown forces and torques F^(k)),
 *   one-body preconditioned with S^(kk)+ and no projection (eq. (2sysprec),
 *   Algorithm 1). */
enum { MFS_MOBILITY = 0, MFS_RESISTANCE = 1 };

/* Factorisation of the one-body blocks (Section 2.3, eq. (pseudo)).
 * MFS_FACTOR_SVD: S_L = U Sigma V^T by rocSOLVER's batched FP64 SVD
 *   (bidiagonal QR); the plan applies S_L^+ = (V Sigma^-1)(U^T .).
 * MFS_FACTOR_QR: S_L = Q R by the library's batched FP64 Householder QR
 *   (blocked, compact WY form: trailing updates on the FP64 matrix cores);
 *   for full column rank S_L^+ = R^-1 Q^T, the same operator, applied in the
 *   same two steps ((R^-1)(Q^T .)), with R^-1 from triangular solves.  A
 *   MFS_MIXED plan applies Q^T in FP32 and R^-1 in FP64 (R^-1 in FP32 would
 *   cost the mixed operator accuracy on smooth inputs).  Much faster to
 *   build; mfs_plan_sizes then reports 1 / (||R||_F ||R^-1||_F), a lower
 *   bound of sigma_min / sigma_max, and the rank check uses that bound.  At
 *   most 8192 columns (3N Stokes, N Laplace) per block. */
enum { MFS_FACTOR_SVD = 0, MFS_FACTOR_QR = 1 };

typedef struct {
    int32_t precision;             /* MFS_MIXED or MFS_FP64: matvec used inside GMRES */
    double mu;                     /* Stokes viscosity (> 0) */
    int64_t n_sys;                 /* number of independent systems (>= 1) */
    const int64_t *sys_body_ptr;   /* [host] [n_sys+1] */
    const int32_t *sys_kind;       /* [host] [n_sys] MFS_LAPLACE or MFS_STOKES */
    const double *centre;          /* [host] [n_body][3] */
    const double *rot;             /* [host] [n_body][3][3] row-major rotation (x = c + R xtilde) */
    const int32_t *shape_of_body;  /* [host] [n_body] */
    int64_t n_shape;
    const int32_t *shape_n_src;    /* [host] [n_shape] N per shape */
    const int32_t *shape_n_trg;    /* [host] [n_shape] M per shape (M >= N) */
    const double *shape_src;       /* [host] concatenated local proxies, sum(N) x 3 */
    const double *shape_trg;       /* [host] concatenated local collocation points, sum(M) x 3 */
    int32_t formulation;           /* MFS_MOBILITY (0, also for a zero-initialised descriptor) or MFS_RESISTANCE */
    int32_t factorization;         /* MFS_FACTOR_SVD (0, the default) or MFS_FACTOR_QR */
} mfs_plan_desc;

/* Builds a plan: uploads geometry, assembles S_L (MFS_MOBILITY) or S^(kk)
 * (MFS_RESISTANCE) for every (shape, kind) in FP64 on the device, factors it
 * (FP64 SVD, or QR with MFS_FACTOR_QR), stores U^T and W = V Sigma^{-1}
 * (Q^T and R^-1) in FP64 and FP32, and the per-body Gram inverses.  Synchronous.  Below, "S_L" stands for the plan's
 * one-body block, and the projection (I - L) is the identity in a
 * MFS_RESISTANCE plan. */
int mfs_plan_create(mfs_plan *out, const mfs_plan_desc *desc, void *stream);
int mfs_plan_destroy(mfs_plan plan);
/* Totals of the three vector layouts above, and the smallest
 * sigma_min/sigma_max over the plan's factors (MFS_FACTOR_QR plans: the
 * smallest 1/(||R||_F ||R^-1||_F), a lower bound of it) ([host] outputs, any
 * may be NULL). */
int mfs_plan_sizes(mfs_plan plan, int64_t *n_gamma, int64_t *n_lambda, int64_t *n_net,
                   double *min_sigma_ratio);
/* Moves the plan's bodies: new centres [host][n_body][3] and rotations
 * [host][n_body][3][3] (same layout as in the descriptor).  S_L, L, K_N and
 * the completion depend only on points relative to their body, so the
 * one-body factors stay (one factorisation per shape serves every congruent
 * body, Sec. 3.3, Remark on congruent bodies); only the world offsets, Gram
 * inverses and pair-operand positions are rebuilt, into the same device
 * buffers (captured matvec graphs stay valid).  The plan then computes exactly
 * what a new plan with these bodies computes.  MFS_EINVAL for NULL or
 * non-finite input.  Synchronous; no work on the plan may be in flight on
 * another stream. */
int mfs_plan_set_bodies(mfs_plan plan, const double *centre, const double *rot, void *stream);

/* Completion strengths and right-hand side (eqs. (al0), (erhsK); (lambda01),
 * (lambda02), (stou0)): s_0 = (q/N) 1 or K_N (K_N^T K_N)^{-1} [f; t] per body,
 * then b = -u_0 with u_0 the pair sum over all pairs of the system, self
 * included.  net [device] in the net layout; b [device] gamma layout;
 * strength0 [device] lambda layout (may be NULL).  prec selects the pair
 * arithmetic of u_0. */
int mfs_rhs(mfs_plan plan, const double *net, double *b, double *strength0, int prec, void *stream);
/* In a MFS_RESISTANCE plan, `net` holds the Dirichlet data per body (net
 * layout): the potential phi^(k), or the rigid velocities [v; omega]; then
 * b = phi^(k) 1_M, or b = K_M U, v + omega x (x_i - c) at every collocation
 * point (eq. (rbm), Section 2.2); no pair sum runs, prec is ignored and
 * strength0 (if given) is set to 0. */

/* Per-body pseudo-inverse blocks (eq. (pseudo); Remark "congruent"):
 *   out = S_L^+ in            (in: gamma layout, out: lambda layout)
 *   flags & MFS_PROJECT:   out = (I - L) S_L^+ in   (MFS_EINVAL in a MFS_RESISTANCE plan)
 *   flags & MFS_TRANSPOSE: out = (S_L^+)^T in   (in: lambda layout, out: gamma
 *                          layout; with PROJECT: (S_L^+)^T (I - L) in)
 * prec selects FP32 MFMA (MFS_MIXED) or FP64 MFMA (MFS_FP64) GEMMs. */
int mfs_precond_apply(mfs_plan plan, const double *in, double *out, int flags, int prec, void *stream);

/* out = A gamma, the square operator of eq. (2esysprec) (gamma and out in the
 * gamma layout, must not alias). */
int mfs_matvec(mfs_plan plan, const double *gamma, double *out, int prec, void *stream);
/* out = A^T w (derived: the paper has no adjoint). */
int mfs_matvec_adjoint(mfs_plan plan, const double *w, double *out, int prec, void *stream);

/* GMRES for A gamma = b (unrestarted per attempt, x0 = 0, classical
 * Gram-Schmidt with reorthogonalisation, Givens rotations, FP64; the
 * least-squares update and the stopping test run on the device, and the host
 * enqueues each iteration before it reads the status of the one before, so
 * the GPU does not wait for it (with a progress callback set it reads every
 * status first; the results are the same).
 * Every system stops on its own when ||r||_2 <= stop_factor tol ||b||_2 (a
 * margin below tol for the outputs' error; see mfs_plan_set_stop_factor).  With
 * a MIXED plan the Krylov matvec is the mixed one; each attempt ends with an
 * FP64 true-residual matvec, and systems whose true residual is above
 * stop_factor tol ||b||_2 restart from their iterate on that residual, each
 * restart reducing it by stop_factor (iterative refinement, at most max_refine
 * restarts).
 * iters [host][n_sys] receives the matvecs spent per system (mixed and FP64),
 * relres [host][n_sys] the final relative residual (the true FP64 one for
 * MIXED plans, the GMRES estimate for FP64 plans); either may be NULL.
 * adjoint != 0 solves A^T gamma = b instead.  Synchronous.
 * Returns MFS_NOT_CONVERGED if some system ends above tol. */
int mfs_gmres_solve(mfs_plan plan, const double *b, double *gamma, double tol, int32_t max_iter,
                    int32_t max_refine, int32_t adjoint, int32_t *iters, double *relres, void *stream);

/* Recovery (Section 3.3; eqs. (vkal), (getU)): lambda = S_L^+ gamma (FP64
 * factors), then out = phi = -mean(alpha) or [v; omega] = -K_N^T lambda per
 * body (net layout).  sigma [device, lambda layout, may be NULL] receives the
 * full strength (I - L) lambda + s_0 (strength0 may be NULL: taken as 0). */
int mfs_extract(mfs_plan plan, const double *gamma, const double *strength0, double *out, double *sigma,
                void *stream);
/* In a MFS_RESISTANCE plan: lambda = S^(kk)+ gamma (Algorithm 1, SOLVE),
 * out = q^(k) = sum_j alpha_j (eq. (qkgauss)) or [f; t] = K_N^T lambda
 * (eq. (force_def)); sigma receives lambda. */

/* Gradients of a loss J(out) through the whole solve, with respect to the
 * body centres and to the given net quantities (charges q, or forces and
 * torques [f; t]).  Bodies move rigidly with their centres; shapes and
 * rotations are held fixed.  Derived from the square system of eq.
 * (2esysprec); the paper has no gradients.
 * Inputs [device]: the forward solution gamma (gamma layout) and strength0
 * (lambda layout, from mfs_rhs), grad_out = dJ/d(out) (net layout).
 * Outputs [device], either may be NULL but not both:
 *   grad_centre [n_body][3]  dJ/dc.  Requires strength0: the pair terms carry
 *                            the full strength (I - L) S_L^+ gamma + s_0.
 *   grad_net    (net layout) dJ/dq or dJ/d[f; t].  The net quantities enter
 *                            only through s_0 (eqs. (al0), (lambda01),
 *                            (lambda02)) in b = -u_0 (eqs. (erhsK), (stou0)):
 *                            grad_net = (1/N) 1^T t (Laplace) or
 *                            (K_N^T K_N)^{-1} K_N^T t (Stokes) with
 *                            t = -sum_k S^(kk')T w^(k), self block included.
 * Work: one adjoint GMRES, A^T w = g with g = (S_L^+)^T dJ/dlambda (the
 * plan's precision; tol, max_iter, max_refine, iters and relres as for
 * mfs_gmres_solve with adjoint = 1), then the backward pair sums over
 * off-body pairs (grad_centre) and one transposed pair sum over all pairs
 * (grad_net).  MFS_EINVAL for a NULL plan, gamma or grad_out, for neither
 * output, for grad_centre without strength0, or for bad tol / max_iter /
 * max_refine; MFS_EUNSUPPORTED in a MFS_RESISTANCE plan.  Returns
 * MFS_NOT_CONVERGED (outputs from the best adjoint iterate) when the adjoint
 * solve ends above tol.  Synchronous. */
int mfs_gmres_solve_backward(mfs_plan plan, const double *gamma, const double *strength0, const double *grad_out,
                             double *grad_centre, double *grad_net, double tol, int32_t max_iter,
                             int32_t max_refine, int32_t *iters, double *relres, void *stream);

/* Surface residual at test points on every body surface, with u the
 * representation of the full strengths sigma [device, lambda layout, e.g. from
 * mfs_extract] over all proxies of the system (same-body pairs included) and
 * motion [device, net layout: the solve's output, or the Dirichlet data of a
 * resistance solve].  Stokes (eq. (residual)): eps(x) = |u(x) - g(x)| / |g(x)|
 * with g = v + omega x (x - c), the body's rigid motion.  Laplace: the
 * absolute error eps(x) = |u(x) - phi| against the body's potential phi, the
 * measure of the elastance convergence study (Sec. 4.1, Fig. f:elastconv(a)).  Test points per shape in the shape frame:
 * shape_n_test [host][n_shape], shape_test [host] concatenated, sum x 3.
 * eps [device] body by body; u_test [device, optional] receives u at the
 * points (3 or 1 values per point).  prec selects the pair arithmetic.
 * Writes the pair-sum source records of the plan (the next matvec rewrites
 * them).  Synchronous. */
int mfs_surface_residual(mfs_plan plan, const double *sigma, const double *motion, const int32_t *shape_n_test,
                         const double *shape_test, double *eps, double *u_test, int prec, void *stream);

/* Instrumentation.  With timing enabled, every pair-sum launch of the plan's
 * matvec (the dominant kernel) is bracketed by HIP events recorded on the
 * call's stream, directly before and after the kernel.  mfs_plan_timing
 * returns, for precision prec, the number of timed launches, their summed
 * kernel time in ms (synchronises on the last recorded event) and the number
 * of off-body pairs one launch evaluates; reset != 0 clears the counters. */
int mfs_plan_set_timing(mfs_plan plan, int32_t enable);
/* Matvecs per system spent by the last mfs_gmres_solve on this plan, split by
 * precision (the Krylov matvecs and the FP64 true-residual checks) [host][n_sys]. */
int mfs_plan_last_solve(mfs_plan plan, int32_t *mixed_matvecs, int32_t *fp64_matvecs);

/* Options.  mfs_plan_set_graph: with enable != 0, mfs_gmres_solve replays the
 * Krylov matvec from a hipGraph, captured on first use per (precision,
 * direction) on a library-owned stream with fixed buffers (the Krylov column
 * is copied into a fixed input first); the captured work holds kernel
 * launches only.  Ignored while timing is enabled.  mfs_plan_autotune: times
 * the matvec pair sum for candidate launch shapes (1 or 2 targets per lane x
 * 1024..16384 work items, which sets the source split x one workgroup per
 * item or a persistent grid of 2048 workgroups claiming items from a queue)
 * on `stream`, reps launches each, and keeps for the forward and transposed
 * sums the shape with the fewest source splits among those within 1.5% of the
 * fastest (timing noise; fewer splits write fewer FP64 slices), reporting it
 * ([host] outputs, may be NULL; *best_tpl is negative for the persistent
 * grid).  Synchronous. */
int mfs_plan_set_graph(mfs_plan plan, int32_t enable);
/* Stopping margin of mfs_gmres_solve (and of the adjoint solve of
 * mfs_gmres_solve_backward): GMRES iterates until its residual (the estimate;
 * in MIXED plans then also the FP64 true residual, by refinement) is at most
 * factor * tol * ||b||_2 per system (Section 4: GMRES with a relative
 * tolerance; factor 1 is that rule as stated), and a solve succeeds when the
 * final relative residual (the FP64 true one for MIXED plans) is at most tol.
 * The relative residual bounds the outputs' error only up to the conditioning
 * of the recovery, so the default, 0.1, keeps U and phi within tol of the
 * exact discrete solution on the benchmark suspensions.  MFS_EINVAL unless
 * 0 < factor <= 1. */
int mfs_plan_set_stop_factor(mfs_plan plan, double factor);
/* Progress of long solves.  With a callback set, mfs_gmres_solve (and the
 * adjoint solve of mfs_gmres_solve_backward) calls it on the calling host thread
 * after every GMRES iteration with: the matvecs spent so far (largest over
 * systems), the number of systems still iterating, and the largest relative
 * residual estimate among the systems of the current attempt.  A non-zero
 * return stops the solve early; it then returns MFS_NOT_CONVERGED with the
 * current iterates.  fn == NULL removes the callback. */
typedef int (*mfs_progress_fn)(void *user, int32_t matvecs, int32_t active_systems, double max_relres);
int mfs_plan_set_progress(mfs_plan plan, mfs_progress_fn fn, void *user);
/* Fixes the launch shape of the plan's pair sums (the choices the autotuner
 * ranges over): targets_per_lane 1 or 2, work_items >= 1 (target blocks x
 * source splits, at least this many), persistent != 0 for the work-queue grid.
 * Synchronous. */
int mfs_plan_set_launch(mfs_plan plan, int32_t targets_per_lane, int32_t work_items, int32_t persistent, void *stream);
int mfs_plan_autotune(mfs_plan plan, int32_t prec, int32_t reps, int32_t *best_tpl, int32_t *best_min_items,
                      double *best_ms, void *stream);
int mfs_plan_timing(mfs_plan plan, int32_t prec, int32_t reset, int64_t *launches, double *total_ms,
                    double *pairs_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* MFS_H */
