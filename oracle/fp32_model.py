"""A float32 model of the mixed-precision steps, used to size the mixed
parity bars.

TEST INFRASTRUCTURE ONLY, like the rest of oracle/: imported by tests/ and by
tests/golden/make_golden.py, never by the GPU library, with which it shares
no code.  It builds on the FP64 oracle (mfs_oracle) and changes only the
precision of the steps named below.

Each function evaluates the oracle's formulas for one step with the operands
a mixed path keeps in FP32 rounded to float32 and the arithmetic done in
float32, and everything the mixed path keeps in FP64 left in FP64:

* pair sums (eqs. (rep), (repS)) and their position gradients: target and
  source offsets from their bodies' reference points, the reference points'
  difference and the strengths rounded to float32; the pair terms in float32;
  runs of 64 consecutive sources summed in float32, the runs in float64;
* pseudo-inverse blocks (eq. (pseudo), Remark "congruent"): the factors U^T
  and W = V Sigma^+ (or U and W^T for the transpose) and the block's input in
  the shape frame rounded to float32, both products in float32, the
  rotations and the projection (I - L) in float64; for a QR plan Q^T (Q) and
  its product in float32, R^-1 (R^-T) and its product in float64.

The model's error against the FP64 oracle on the same input is the size of
the error that FP32 storage and arithmetic of these steps cause on that
input; a mixed GPU result does the same roundings in another order, so its
error is of the same size.  The mixed bars are a fixed multiple of it.

The same functions with dt = float64 model an FP64 path: the same formulas
in float64 with another summation order than the oracle's (runs of 64), and
the pseudo-inverse from a backward-stable FP64 factorisation of S_L, the
exact factorisation of a block within u64 |S_L|_2 of it (see _factors).
The FP64 bars are the same multiple of that model's error.
"""
from __future__ import annotations

import numpy as np

from . import mfs_oracle as O

F32 = np.float32
RUN = 64
BAR_FACTOR = 4.0  # bar = BAR_FACTOR x the model's error (rounding order differs)


def _f32(a, dt=F32):
    return np.asarray(a, dtype=dt)


def ref_first_source(n_body, src_body, Y, trg_body=None, X=None):
    """Reference point of each body as the standalone entry points take it: its
    first source point (its first target point when it has no source)."""
    ref = np.zeros((n_body, 3))
    if trg_body is not None:
        for i in range(len(trg_body) - 1, -1, -1):
            ref[trg_body[i]] = X[i]
    for j in range(len(src_body) - 1, -1, -1):
        ref[src_body[j]] = Y[j]
    return ref


def _blocks(n_rows, n_src, budget=48_000_000):
    step = max(1, budget // max(1, 3 * n_src))
    for a in range(0, n_rows, step):
        yield a, min(n_rows, a + step)


def _run_sum(t):
    """t (rows, n_src, ...): runs of RUN sources summed in t's precision, then float64."""
    r, n = t.shape[0], t.shape[1]
    pad = (-n) % RUN
    if pad:
        t = np.concatenate([t, np.zeros((r, pad) + t.shape[2:], t.dtype)], axis=1)
    runs = t.reshape((r, -1, RUN) + t.shape[2:]).sum(axis=2, dtype=t.dtype)
    return runs.sum(axis=1, dtype=np.float64)


def _pair_d(X, tb, Y, sb, ref, rows, dt=F32):
    """d = (round(c_t - c_s) + xt) - ys in precision dt for target rows a:b against every source."""
    xt = _f32(X[rows] - ref[tb[rows]], dt)
    ys = _f32(Y - ref[sb], dt)
    dc = _f32(ref[tb[rows]][:, None, :] - ref[sb][None, :, :], dt)
    return (dc + xt[:, None, :]) - ys[None, :, :]


def pair_sum(kind, X, tb, Y, sb, s, ref, skip=True, mu=1.0, dt=F32):
    """u_i = sum_j G(x_i - y_j) s_j in the model of precision dt (ref: (n_body, 3)
    reference points; tb, sb: body ids)."""
    X, Y, tb, sb = np.asarray(X), np.asarray(Y), np.asarray(tb), np.asarray(sb)
    sv = _f32(s, dt)
    out = np.zeros((X.shape[0], 3) if kind == O.STOKES else X.shape[0])
    c = dt(1.0 / (8.0 * np.pi * mu)) if kind == O.STOKES else dt(1.0 / (4.0 * np.pi))
    for a, b in _blocks(X.shape[0], Y.shape[0]):
        rows = slice(a, b)
        d = _pair_d(X, tb, Y, sb, ref, rows, dt)
        rinv = dt(1.0) / np.sqrt((d * d).sum(axis=-1, dtype=dt))
        if skip:
            rinv = np.where(tb[rows][:, None] == sb[None, :], dt(0.0), rinv)
        if kind == O.LAPLACE:
            t = (sv[None, :] * rinv) * c
        else:
            ds = (d * sv[None, :, :]).sum(axis=-1, dtype=dt)
            t = (sv[None, :, :] + d * (ds * rinv * rinv)[..., None]) * (rinv * c)[..., None]
        out[rows] = _run_sum(t)
    return out


def pair_grad(kind, X, tb, w, Y, sb, s, ref, skip=True, mu=1.0, dt=F32):
    """Position gradients of Phi = sum w_i . G(x_i - y_j) s_j in the model of
    precision dt: (dPhi/dx_i, dPhi/dy_j)."""
    X, Y, tb, sb = np.asarray(X), np.asarray(Y), np.asarray(tb), np.asarray(sb)
    wv_all, sv_all = _f32(w, dt), _f32(s, dt)

    def lanes(LX, lb, lw, SY, sbb, ss, sign):
        g = np.zeros((LX.shape[0], 3))
        for a, b in _blocks(LX.shape[0], SY.shape[0]):
            rows = slice(a, b)
            d = sign * _pair_d(LX, lb, SY, sbb, ref, rows, dt)  # d = x - y
            r2 = (d * d).sum(axis=-1, dtype=dt)
            rinv = dt(1.0) / np.sqrt(r2)
            if skip:
                rinv = np.where(lb[rows][:, None] == sbb[None, :], dt(0.0), rinv)
            r3 = rinv * rinv * rinv
            if kind == O.LAPLACE:
                cst = dt(-1.0 / (4.0 * np.pi))
                t = d * (cst * lw[rows][:, None] * ss[None, :] * r3)[..., None]
            else:
                cst = dt(1.0 / (8.0 * np.pi * mu))
                wv = lw[rows][:, None, :]
                sv = ss[None, :, :]
                ws = (wv * sv).sum(axis=-1, dtype=dt)
                wd = (wv * d).sum(axis=-1, dtype=dt)
                sd = (sv * d).sum(axis=-1, dtype=dt)
                t = (-ws[..., None] * d + wd[..., None] * sv + sd[..., None] * wv
                     - (dt(3.0) * wd * sd * rinv * rinv)[..., None] * d) * (cst * r3)[..., None]
            g[rows] = sign * _run_sum(t)
        return g

    gx = lanes(X, tb, wv_all, Y, sb, sv_all, dt(1.0))
    gy = lanes(Y, sb, sv_all, X, tb, wv_all, dt(-1.0))
    return gx, gy


FIELD_PRESSURE, FIELD_TRACTION, FIELD_LAPLACE_GRADIENT = 0, 1, 2


def field(kind_field, X, tb, Y, sb, s, ref, normal=None, skip=False, dt=F32):
    """Derived fields of the representation in the model of precision dt: Stokes
    pressure (1/(8 pi)) sum 2 d.f / r^3, traction -(3/(4 pi)) sum d (d.n)(d.f) / r^5,
    Laplace gradient -(1/(4 pi)) sum q d / r^3."""
    X, Y, tb, sb = np.asarray(X), np.asarray(Y), np.asarray(tb), np.asarray(sb)
    sv = _f32(s, dt)
    nv = _f32(normal, dt) if normal is not None else None
    out = np.zeros(X.shape[0]) if kind_field == FIELD_PRESSURE else np.zeros((X.shape[0], 3))
    for a, b in _blocks(X.shape[0], Y.shape[0]):
        rows = slice(a, b)
        d = _pair_d(X, tb, Y, sb, ref, rows, dt)
        rinv = dt(1.0) / np.sqrt((d * d).sum(axis=-1, dtype=dt))
        if skip:
            rinv = np.where(tb[rows][:, None] == sb[None, :], dt(0.0), rinv)
        r3 = rinv * rinv * rinv
        if kind_field == FIELD_PRESSURE:
            t = (d * sv[None, :, :]).sum(axis=-1, dtype=dt) * r3 * dt(1.0 / (4.0 * np.pi))
        elif kind_field == FIELD_TRACTION:
            df = (d * sv[None, :, :]).sum(axis=-1, dtype=dt)
            dn = (d * nv[rows][:, None, :]).sum(axis=-1, dtype=dt)
            t = d * (dt(-3.0 / (4.0 * np.pi)) * df * dn * r3 * rinv * rinv)[..., None]
        else:
            t = d * (dt(-1.0 / (4.0 * np.pi)) * sv[None, :] * r3)[..., None]
        out[rows] = _run_sum(t)
    return out


def surface_residual(pr, sigma, out, test_local, dt=F32):
    """The surface residual of eq. (residual) as Problem.surface_residual
    computes it, with the representation's pair sum (all proxies, self
    included) in the model of precision dt."""
    pts, ids = [], []
    for k, b in enumerate(pr.bodies):
        pts.append(b.centre + np.asarray(test_local) @ b.rot.T)
        ids.append(np.full(len(test_local), k, np.int32))
    Xt, tb = np.concatenate(pts), np.concatenate(ids)
    s = sigma.reshape(-1, 3) if pr.kind == O.STOKES else sigma
    u = pair_sum(pr.kind, Xt, tb, pr.Y, pr.src_body, s, _centres(pr), False, pr.mu, dt)
    out = np.asarray(out, np.float64)
    if pr.kind == O.LAPLACE:
        return np.abs(u - out[tb])
    c = np.stack([pr.bodies[k].centre for k in tb])
    g = out[tb, :3] + np.cross(out[tb, 3:], Xt - c)
    return np.linalg.norm(u - g, axis=1) / np.linalg.norm(g, axis=1)


# ---------------------------------------------------------------------------
# pseudo-inverse blocks, operator, right-hand side (a Problem from the oracle)
# ---------------------------------------------------------------------------

def _block_matrix(pr, key):
    """The block that factor `key` factors: a body's own S_L, or its shape's in the body frame."""
    if pr.per_body:
        return pr.S_L(key)
    sh = pr.shapes[key]
    return pr.one_body_matrix(sh.trg, sh.src, np.zeros(3))


def _factors(pr, F, key, qr, dt=F32):
    """The two factors a plan applies S_L^+ with, in precision dt: U^T and
    W = V Sigma^+ of the SVD (and U, W^T for the transpose), or, for a QR plan
    (S_L = Q R, full column rank), Q^T and R^-1 (and Q, R^-T).

    float32: the oracle's SVD factors (or a QR of the same block) rounded;
    a mixed QR plan rounds Q^T and Q only and applies R^-1 in FP64 (the
    product's input is then the FP32 result of the first step).
    float64: the factors of a backward-stable FP64 factorisation, i.e. the
    exact SVD (or QR) of a block within u64 |S_L|_2 of S_L: S_L + E with
    E = u64 |S_L|_2 Z / |Z|_2, Z a seeded Gaussian matrix (|Z|_2 taken as
    sqrt(rows) + sqrt(cols), its size for large Gaussian matrices).  A block
    assembled and factored in FP64 by another order of operations differs
    from the oracle's in this way; its pseudo-inverse differs by about
    u64 cond(S_L)."""
    tag = ("_qr" if qr else "_m") + ("32" if dt == F32 else "64")
    if hasattr(F, tag):
        return getattr(F, tag)
    if qr and pr.per_body:
        raise ValueError("the QR model factors per shape")
    if dt == F32 and not qr:
        fac = (F.U.T, F.Vt.T / F.s, F.U, (F.Vt.T / F.s).T)
    else:
        S = _block_matrix(pr, key)
        if dt != F32:
            Z = np.random.default_rng(np.random.SeedSequence([7919, int(key)])).standard_normal(S.shape)
            S = S + (np.finfo(np.float64).eps / 2) * F.s[0] * Z / (np.sqrt(S.shape[0]) + np.sqrt(S.shape[1]))
        if qr:
            Q, R = np.linalg.qr(S)
            Ri = np.linalg.inv(R)
            fac = (Q.T, Ri, Q, Ri.T)
        else:
            U, sv, Vt = np.linalg.svd(S, full_matrices=False)
            fac = (U.T, Vt.T / sv, U, (Vt.T / sv).T)
    if qr and dt == F32:  # a mixed QR plan keeps R^-1 in FP64 (Q^T and Q in FP32)
        fac = tuple(np.ascontiguousarray(_f32(m, F32 if i in (0, 2) else np.float64)) for i, m in enumerate(fac))
    else:
        fac = tuple(np.ascontiguousarray(_f32(m, dt)) for m in fac)
    setattr(F, tag, fac)
    return fac


def pinv_apply(pr, k, v, transpose=False, qr=False, dt=F32):
    """S_L^(k)+ v (or its transpose) with factors and products in precision dt
    (qr: the factors of a QR plan)."""
    b = pr.bodies[k]
    F = pr.factors[b.factor_key]
    Ut, Wm, U, Wt = _factors(pr, F, b.factor_key, qr, dt)
    rot = pr.kind == O.STOKES and not pr.per_body
    x = pr._rotate(b.rot, v, transpose=True) if rot else np.asarray(v)
    if transpose and qr and dt == F32:  # R^-T x in FP64, rounded, then Q in FP32
        y = (U @ (Wt @ np.asarray(x, np.float64)).astype(F32)).astype(np.float64)
    elif transpose:
        y = (U @ (Wt @ _f32(x, dt))).astype(np.float64)
    else:
        y = (Wm @ (Ut @ _f32(x, dt))).astype(np.float64)
    return pr._rotate(b.rot, y) if rot else y


def _centres(pr):
    return np.stack([b.centre for b in pr.bodies])


def precondition(pr, gamma, project=True, qr=False, dt=F32):
    """(I - L^(k)) S_L^(k)+ gamma^(k) for every body (the bodies sharing a factor
    as the columns of one product in precision dt, as a plan applies them)."""
    groups = {}
    for k, b in enumerate(pr.bodies):
        groups.setdefault(b.factor_key, []).append(k)
    rot = pr.kind == O.STOKES and not pr.per_body
    lam = [None] * len(pr.bodies)
    for key, ks in groups.items():
        Ut, Wm, _, _ = _factors(pr, pr.factors[key], key, qr, dt)
        cols = [pr._rotate(pr.bodies[k].rot, pr.gblock(gamma, k), transpose=True) if rot else pr.gblock(gamma, k)
                for k in ks]
        Y = (Wm @ (Ut @ _f32(np.stack(cols, axis=1), dt))).astype(np.float64)
        for j, k in enumerate(ks):
            lam[k] = pr._rotate(pr.bodies[k].rot, Y[:, j]) if rot else Y[:, j]
    return np.concatenate([pr.project(k, lam[k]) if project else lam[k] for k in range(len(pr.bodies))])


def matvec(pr, gamma, rows=None, qr=False, dt=F32):
    """(A gamma)^(k) of eq. (2esysprec) (or (2sysprec) for a ResistanceProblem)."""
    beta = precondition(pr, gamma, qr=qr, dt=dt)
    s = beta.reshape(-1, 3) if pr.kind == O.STOKES else beta
    X, tb = (pr.X, pr.trg_body) if rows is None else (pr.X[rows], pr.trg_body[rows])
    u = pair_sum(pr.kind, X, tb, pr.Y, pr.src_body, s, _centres(pr), True, pr.mu, dt).reshape(-1)
    idx = slice(None) if rows is None else pr._row_index(rows)
    return np.asarray(gamma)[idx] + u


def matvec_T(pr, w, qr=False, dt=F32):
    """(A^T w)^(k') = w^(k') + (S_L^(k')+)^T (I - L^(k')) sum_{k != k'} S^(kk')T w^(k)."""
    ws = w.reshape(-1, 3) if pr.kind == O.STOKES else w
    t = pair_sum(pr.kind, pr.Y, pr.src_body, pr.X, pr.trg_body, ws, _centres(pr), True, pr.mu, dt).reshape(-1)
    out = [pinv_apply(pr, k, pr.project(k, pr.sblock(t, k)), transpose=True, qr=qr, dt=dt)
           for k in range(len(pr.bodies))]
    return w + np.concatenate(out)


def rhs(pr, net, rows=None, dt=F32):
    """b = -u_0 with s_0 from the oracle's completion (FP64 on both paths) and
    the all-pairs sum in the model of precision dt."""
    s0 = pr.completion_strengths(net)
    s = s0.reshape(-1, 3) if pr.kind == O.STOKES else s0
    X, tb = (pr.X, pr.trg_body) if rows is None else (pr.X[rows], pr.trg_body[rows])
    return -pair_sum(pr.kind, X, tb, pr.Y, pr.src_body, s, _centres(pr), False, pr.mu, dt).reshape(-1)


def precond_apply(pr, v, transpose=False, project=False, qr=False, dt=F32):
    """The blocks as mfs_precond_apply applies them: S_L^+ v, (I - L) S_L^+ v,
    (S_L^+)^T v or (S_L^+)^T (I - L) v, per body."""
    out = []
    for k in range(len(pr.bodies)):
        if transpose:
            x = pr.sblock(v, k)
            out.append(pinv_apply(pr, k, pr.project(k, x) if project else x, transpose=True, qr=qr, dt=dt))
        else:
            lam = pinv_apply(pr, k, pr.gblock(v, k), qr=qr, dt=dt)
            out.append(pr.project(k, lam) if project else lam)
    return np.concatenate(out)


def bar(model_err: float, floor: float = 1e-15) -> float:
    """The bar for a step whose model errs by model_err."""
    return BAR_FACTOR * max(model_err, floor)


# GMRES stopping margin of the library (mfs_plan_set_stop_factor default)
STOP = 0.1


def extract(pr, gamma, s0, qr=False, dt=np.float64):
    """pr.extract (eqs. (vkal), (getU)) with the model's pseudo-inverse factors
    of precision dt in place of the oracle's."""
    pr.pinv_apply = lambda k, v: pinv_apply(pr, k, v, qr=qr, dt=dt)
    try:
        return pr.extract(gamma, s0)
    finally:
        del pr.pinv_apply


def solve_bars(pr, net, tol, ref=None, keys=("out",), cap=None, qr=False, dt=F32, gamma=None, stop=STOP):
    """Bars for the outputs of a solve at GMRES tol `tol` whose operator is
    applied in precision dt (float32: a mixed solve; float64: an FP64 one).

    Two limits, the larger of which sets the bar (times BAR_FACTOR, capped:
    1e-5 for the outputs the method reports):
    * the stopping residual: GMRES iterates until its estimate is at most
      stop * tol; the FP64 true residual then carries the operator's own error
      too (eps_mv, the model's matvec error on a random vector), and a system
      above tol restarts from its iterate (refinement) until the true residual
      is at most tol.  So the solve ends at a residual of at most
      r = min(tol, max(stop * tol, eps_mv)).  The oracle's GMRES iterates
      around r (the first with residual at most r, and the one before it)
      give the ratio of output error to relative residual near convergence:
      this limit is the larger ratio x r;
    * the operator: its matvecs cannot tell the solution gamma from
      gamma + delta, delta = (A_model - A) gamma the model's matvec error at
      the solution, so the outputs are known only up to what delta does to
      them through the recovery (S_L^+ with FP64 factors, eqs. (vkal),
      (getU); for dt = float64 the model's own backward-stable FP64
      factors, which differ from the oracle's as the path's do): this limit is
      the change of each output under gamma + delta.
    stop: the plan's stopping factor (mfs_plan_set_stop_factor; STOP unless
    the plan sets another).
    gamma: the solution under test (a host array), when it is known: the
    returned dict then also carries its residual under the oracle's b and A,
    rho_t = |b - A gamma|_2 / |b|_2 ("residual"), and the most that residual
    may be ("residual_bound"): the library's check holds the residual against
    its own right-hand side to tol, so rho_t <= tol + |b_path - b|_2 / |b|_2,
    the second term 4 x the model's right-hand-side error (FP32 pair sums in
    a mixed plan's b; FP64 rounding otherwise).  The bars themselves do not
    depend on gamma.
    ref: the oracle's solve at a tight tolerance (a dict as Problem.solve
    returns; solved here when None).  For dt = float64, r is close to the
    tolerance such a reference is solved at, so the reference is solved here
    at r / 100 whatever is passed."""
    fp64 = dt == np.float64
    g = np.random.default_rng(np.random.SeedSequence(9999)).standard_normal(pr.n_gamma)
    ref_mv = pr.matvec(g)
    eps_mv = float(np.abs(matvec(pr, g, qr=qr, dt=dt) - ref_mv).max() / np.abs(ref_mv).max())
    r = min(tol, max(stop * tol, eps_mv))
    rho_t = None
    if gamma is not None:
        b, _ = pr.rhs(net)
        bn = np.linalg.norm(b)
        rho_t = float(np.linalg.norm(b - pr.matvec(np.asarray(gamma, np.float64))) / bn)
        b_model = dirichlet_data(pr, net) if isinstance(pr, O.ResistanceProblem) else rhs(pr, net, dt=dt)
        rho_bound = tol + BAR_FACTOR * max(float(np.linalg.norm(b_model - b) / bn), 1e-15)
    if fp64:
        ref = pr.solve(net, tol=max(1e-2 * r, 1e-15))
    elif ref is None or "gamma" not in ref:
        ref = pr.solve(net, tol=1e-13)
    # the oracle's iterate at r and the one before it (residual above r): the
    # ratio is taken from both, as the last step may overshoot r by orders of
    # magnitude and land on the reference itself
    sol = pr.solve(net, tol=r)
    its = [(sol, max(float(sol["hist"][-1]), 1e-300))]
    if sol["iters"] >= 1:
        prev = pr.solve(net, tol=r, max_iter=sol["iters"] - 1)
        its.append((prev, max(float(prev["hist"][-1]), 1e-300)))
    gam = np.asarray(ref["gamma"])
    delta = matvec(pr, gam, qr=qr, dt=dt) - pr.matvec(gam)
    moved_out = extract(pr, gam + delta, ref["s0"], qr, dt) if fp64 else pr.extract(gam + delta, ref["s0"])
    moved = dict(zip(("out", "lam", "sigma"), moved_out))
    moved["gamma"] = gam + delta
    out = {}
    for k in keys:
        den = np.abs(np.asarray(ref[k])).max()
        ratio = max(np.abs(np.asarray(it[k]) - np.asarray(ref[k])).max() / den / rho for it, rho in its)
        floor = np.abs(np.asarray(moved[k]) - np.asarray(ref[k])).max() / den
        b = bar(max(ratio * r, floor))
        out[k] = min(b, cap) if cap else b
    if rho_t is not None:
        out["residual"] = rho_t
        out["residual_bound"] = rho_bound
    return out


def gradient_bars(pr, net, tol, dt=F32, cap=1e-5):
    """Bars for dJ/dc and dJ/d(net) of J = sum |U|^2 (or sum phi^2) from a
    solve and an adjoint solve, both at GMRES tol `tol`, on a path whose pair
    sums run in precision dt.  Each is 4 x (the model's error of the pair sums
    that form the gradient, taken on the oracle's own adjoint solution and
    strengths + the oracle's own error when both its solves stop at `tol`;
    the adjoint's data 2U carries the forward solve's error, so tol itself
    and not the stopping residual below it sizes that part), at most `cap`.
    Returns (oracle gradient at tol 1e-14, its info dict,
    {"centre": bar, "net": bar})."""
    _, g_ref, info = pr.velocity_loss_gradient(net, tol=1e-14)
    _, g_tol, info_tol = pr.velocity_loss_gradient(net, tol=tol)
    shape = (-1, 3) if pr.kind == O.STOKES else (-1,)
    w, sg = info["w"].reshape(shape), info["sol"]["sigma"].reshape(shape)
    cen = _centres(pr)
    mgx, mgy = pair_grad(pr.kind, pr.X, pr.trg_body, w, pr.Y, pr.src_body, sg, cen, True, pr.mu, dt)
    gm = np.zeros((len(pr.bodies), 3))
    np.add.at(gm, pr.trg_body, mgx)
    np.add.at(gm, pr.src_body, mgy)
    # dJ/d(net): the transposed all-pairs sum of w, reduced per body as the oracle does
    t = -pair_sum(pr.kind, pr.Y, pr.src_body, pr.X, pr.trg_body, w, cen, False, pr.mu, dt).reshape(-1)
    gn = []
    for k, b in enumerate(pr.bodies):
        tk = pr.sblock(t, k)
        if pr.kind == O.LAPLACE:
            gn.append(np.mean(tk))
        else:
            KN = O.K_matrix(b.Y, b.centre)
            gn.append(np.linalg.solve(KN.T @ KN, KN.T @ tk))
    gn_ref = np.asarray(info["grad_net"])

    def rel(a, r):
        return float(np.abs(np.asarray(a) - r).max() / np.abs(r).max())
    bars = {"centre": min(cap, bar(rel(-gm, g_ref) + rel(g_tol, g_ref))),
            "net": min(cap, bar(rel(np.array(gn), gn_ref) + rel(info_tol["grad_net"], gn_ref)))}
    return g_ref, info, bars


def dirichlet_data(pr, data):
    """The Dirichlet data of a ResistanceProblem (phi 1, or v + omega x
    (x_i - c), eq. (rbm)) with the offsets x_i - c taken as R x~_i from the
    shape's body-frame points, without the round trip through world
    coordinates.  FP64 throughout: its difference from the oracle's data is
    the rounding of that round trip, the size of the difference two FP64
    evaluations of the data may show."""
    data = np.asarray(data, np.float64)
    out = []
    for k, b in enumerate(pr.bodies):
        if pr.kind == O.LAPLACE:
            out.append(np.full(b.X.shape[0], data[k]))
            continue
        off = pr.shapes[b.factor_key].trg @ b.rot.T if not pr.per_body else b.X - b.centre
        out.append(O.K_matrix(off, np.zeros(3)) @ data[k])
    return np.concatenate(out)
