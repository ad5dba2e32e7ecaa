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
  and W = V Sigma^+ (or U and W^T for the transpose; Q^T and R^-1 for a QR
  plan) and the block's input in the shape frame rounded to float32, both
  products in float32, the rotations and the projection (I - L) in float64.

The model's error against the FP64 oracle on the same input is the size of
the error that FP32 storage and arithmetic of these steps cause on that
input; a mixed GPU result does the same roundings in another order, so its
error is of the same size.  The mixed bars are a fixed multiple of it.
"""
from __future__ import annotations

import numpy as np

from . import mfs_oracle as O

F32 = np.float32
RUN = 64
BAR_FACTOR = 4.0  # bar = BAR_FACTOR x the model's error (rounding order differs)


def _f32(a):
    return np.asarray(a, dtype=F32)


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
    """t (rows, n_src, ...) float32: runs of RUN sources summed in float32, then float64."""
    r, n = t.shape[0], t.shape[1]
    pad = (-n) % RUN
    if pad:
        t = np.concatenate([t, np.zeros((r, pad) + t.shape[2:], F32)], axis=1)
    runs = t.reshape((r, -1, RUN) + t.shape[2:]).sum(axis=2, dtype=F32)
    return runs.sum(axis=1, dtype=np.float64)


def _pair_d(X, tb, Y, sb, ref, rows):
    """d = (float(c_t - c_s) + xt) - ys in float32 for target rows a:b against every source."""
    xt = _f32(X[rows] - ref[tb[rows]])
    ys = _f32(Y - ref[sb])
    dc = _f32(ref[tb[rows]][:, None, :] - ref[sb][None, :, :])
    return (dc + xt[:, None, :]) - ys[None, :, :]


def pair_sum(kind, X, tb, Y, sb, s, ref, skip=True, mu=1.0):
    """u_i = sum_j G(x_i - y_j) s_j in the float32 model (ref: (n_body, 3)
    reference points; tb, sb: body ids)."""
    X, Y, tb, sb = np.asarray(X), np.asarray(Y), np.asarray(tb), np.asarray(sb)
    s32 = _f32(s)
    out = np.zeros((X.shape[0], 3) if kind == O.STOKES else X.shape[0])
    c = F32(1.0 / (8.0 * np.pi * mu)) if kind == O.STOKES else F32(1.0 / (4.0 * np.pi))
    for a, b in _blocks(X.shape[0], Y.shape[0]):
        rows = slice(a, b)
        d = _pair_d(X, tb, Y, sb, ref, rows)
        rinv = F32(1.0) / np.sqrt((d * d).sum(axis=-1, dtype=F32))
        if skip:
            rinv = np.where(tb[rows][:, None] == sb[None, :], F32(0.0), rinv)
        if kind == O.LAPLACE:
            t = (s32[None, :] * rinv) * c
        else:
            ds = (d * s32[None, :, :]).sum(axis=-1, dtype=F32)
            t = (s32[None, :, :] + d * (ds * rinv * rinv)[..., None]) * (rinv * c)[..., None]
        out[rows] = _run_sum(t)
    return out


def pair_grad(kind, X, tb, w, Y, sb, s, ref, skip=True, mu=1.0):
    """Position gradients of Phi = sum w_i . G(x_i - y_j) s_j in the float32
    model: (dPhi/dx_i, dPhi/dy_j)."""
    X, Y, tb, sb = np.asarray(X), np.asarray(Y), np.asarray(tb), np.asarray(sb)
    w32, s32 = _f32(w), _f32(s)

    def lanes(LX, lb, lw, SY, sbb, ss, sign):
        g = np.zeros((LX.shape[0], 3))
        for a, b in _blocks(LX.shape[0], SY.shape[0]):
            rows = slice(a, b)
            d = sign * _pair_d(LX, lb, SY, sbb, ref, rows)  # d = x - y
            r2 = (d * d).sum(axis=-1, dtype=F32)
            rinv = F32(1.0) / np.sqrt(r2)
            if skip:
                rinv = np.where(lb[rows][:, None] == sbb[None, :], F32(0.0), rinv)
            r3 = rinv * rinv * rinv
            if kind == O.LAPLACE:
                cst = F32(-1.0 / (4.0 * np.pi))
                t = d * (cst * lw[rows][:, None] * ss[None, :] * r3)[..., None]
            else:
                cst = F32(1.0 / (8.0 * np.pi * mu))
                wv = lw[rows][:, None, :]
                sv = ss[None, :, :]
                ws = (wv * sv).sum(axis=-1, dtype=F32)
                wd = (wv * d).sum(axis=-1, dtype=F32)
                sd = (sv * d).sum(axis=-1, dtype=F32)
                t = (-ws[..., None] * d + wd[..., None] * sv + sd[..., None] * wv
                     - (F32(3.0) * wd * sd * rinv * rinv)[..., None] * d) * (cst * r3)[..., None]
            g[rows] = sign * _run_sum(t)
        return g

    gx = lanes(X, tb, w32, Y, sb, s32, F32(1.0))
    gy = lanes(Y, sb, s32, X, tb, w32, F32(-1.0))
    return gx, gy


FIELD_PRESSURE, FIELD_TRACTION, FIELD_LAPLACE_GRADIENT = 0, 1, 2


def field(kind_field, X, tb, Y, sb, s, ref, normal=None, skip=False):
    """Derived fields of the representation in the float32 model: Stokes
    pressure (1/(8 pi)) sum 2 d.f / r^3, traction -(3/(4 pi)) sum d (d.n)(d.f) / r^5,
    Laplace gradient -(1/(4 pi)) sum q d / r^3."""
    X, Y, tb, sb = np.asarray(X), np.asarray(Y), np.asarray(tb), np.asarray(sb)
    s32 = _f32(s)
    n32 = _f32(normal) if normal is not None else None
    out = np.zeros(X.shape[0]) if kind_field == FIELD_PRESSURE else np.zeros((X.shape[0], 3))
    for a, b in _blocks(X.shape[0], Y.shape[0]):
        rows = slice(a, b)
        d = _pair_d(X, tb, Y, sb, ref, rows)
        rinv = F32(1.0) / np.sqrt((d * d).sum(axis=-1, dtype=F32))
        if skip:
            rinv = np.where(tb[rows][:, None] == sb[None, :], F32(0.0), rinv)
        r3 = rinv * rinv * rinv
        if kind_field == FIELD_PRESSURE:
            t = (d * s32[None, :, :]).sum(axis=-1, dtype=F32) * r3 * F32(1.0 / (4.0 * np.pi))
        elif kind_field == FIELD_TRACTION:
            df = (d * s32[None, :, :]).sum(axis=-1, dtype=F32)
            dn = (d * n32[rows][:, None, :]).sum(axis=-1, dtype=F32)
            t = d * (F32(-3.0 / (4.0 * np.pi)) * df * dn * r3 * rinv * rinv)[..., None]
        else:
            t = d * (F32(-1.0 / (4.0 * np.pi)) * s32[None, :] * r3)[..., None]
        out[rows] = _run_sum(t)
    return out


def surface_residual(pr, sigma, out, test_local):
    """The surface residual of eq. (residual) as Problem.surface_residual
    computes it, with the representation's pair sum (all proxies, self
    included) in the float32 model."""
    pts, ids = [], []
    for k, b in enumerate(pr.bodies):
        pts.append(b.centre + np.asarray(test_local) @ b.rot.T)
        ids.append(np.full(len(test_local), k, np.int32))
    Xt, tb = np.concatenate(pts), np.concatenate(ids)
    s = sigma.reshape(-1, 3) if pr.kind == O.STOKES else sigma
    u = pair_sum(pr.kind, Xt, tb, pr.Y, pr.src_body, s, _centres(pr), False, pr.mu)
    out = np.asarray(out, np.float64)
    if pr.kind == O.LAPLACE:
        return np.abs(u - out[tb])
    c = np.stack([pr.bodies[k].centre for k in tb])
    g = out[tb, :3] + np.cross(out[tb, 3:], Xt - c)
    return np.linalg.norm(u - g, axis=1) / np.linalg.norm(g, axis=1)


# ---------------------------------------------------------------------------
# pseudo-inverse blocks, operator, right-hand side (a Problem from the oracle)
# ---------------------------------------------------------------------------

def _factor32(pr, F, key, qr):
    """The two factors a mixed plan keeps in FP32: U^T and W = V Sigma^+ of the
    SVD (and U, W^T for the transpose), or, for a QR plan (S_L = Q R, full
    column rank), Q^T and R^-1 (and Q, R^-T)."""
    if qr:
        if not hasattr(F, "_qr32"):
            sh = pr.shapes[key]
            Q, R = np.linalg.qr(pr.one_body_matrix(sh.trg, sh.src, np.zeros(3)))
            Ri = np.linalg.inv(R)
            F._qr32 = (_f32(Q.T), _f32(Ri), _f32(Q), _f32(Ri.T))
        return F._qr32
    if not hasattr(F, "_m32"):
        F._m32 = (_f32(F.U.T), _f32(F.Vt.T / F.s), _f32(F.U), _f32((F.Vt.T / F.s).T))
    return F._m32


def pinv_apply(pr, k, v, transpose=False, qr=False):
    """S_L^(k)+ v (or its transpose) with float32 factors and products (qr: the
    factors of a QR plan)."""
    b = pr.bodies[k]
    F = pr.factors[b.factor_key]
    if qr and pr.per_body:
        raise ValueError("the QR model factors per shape")
    Ut, Wm, U, Wt = _factor32(pr, F, b.factor_key, qr)
    rot = pr.kind == O.STOKES and not pr.per_body
    x = pr._rotate(b.rot, v, transpose=True) if rot else np.asarray(v)
    if transpose:
        y = (U @ (Wt @ _f32(x))).astype(np.float64)
    else:
        y = (Wm @ (Ut @ _f32(x))).astype(np.float64)
    return pr._rotate(b.rot, y) if rot else y


def _centres(pr):
    return np.stack([b.centre for b in pr.bodies])


def precondition(pr, gamma, project=True, qr=False):
    """(I - L^(k)) S_L^(k)+ gamma^(k) for every body (the bodies sharing a factor
    as the columns of one float32 product, as a plan applies them)."""
    groups = {}
    for k, b in enumerate(pr.bodies):
        groups.setdefault(b.factor_key, []).append(k)
    rot = pr.kind == O.STOKES and not pr.per_body
    lam = [None] * len(pr.bodies)
    for key, ks in groups.items():
        Ut, Wm, _, _ = _factor32(pr, pr.factors[key], key, qr)
        cols = [pr._rotate(pr.bodies[k].rot, pr.gblock(gamma, k), transpose=True) if rot else pr.gblock(gamma, k)
                for k in ks]
        Y = (Wm @ (Ut @ _f32(np.stack(cols, axis=1)))).astype(np.float64)
        for j, k in enumerate(ks):
            lam[k] = pr._rotate(pr.bodies[k].rot, Y[:, j]) if rot else Y[:, j]
    return np.concatenate([pr.project(k, lam[k]) if project else lam[k] for k in range(len(pr.bodies))])


def matvec(pr, gamma, rows=None, qr=False):
    """(A gamma)^(k) of eq. (2esysprec) (or (2sysprec) for a ResistanceProblem)."""
    beta = precondition(pr, gamma, qr=qr)
    s = beta.reshape(-1, 3) if pr.kind == O.STOKES else beta
    X, tb = (pr.X, pr.trg_body) if rows is None else (pr.X[rows], pr.trg_body[rows])
    u = pair_sum(pr.kind, X, tb, pr.Y, pr.src_body, s, _centres(pr), True, pr.mu).reshape(-1)
    idx = slice(None) if rows is None else pr._row_index(rows)
    return np.asarray(gamma)[idx] + u


def matvec_T(pr, w):
    """(A^T w)^(k') = w^(k') + (S_L^(k')+)^T (I - L^(k')) sum_{k != k'} S^(kk')T w^(k)."""
    ws = w.reshape(-1, 3) if pr.kind == O.STOKES else w
    t = pair_sum(pr.kind, pr.Y, pr.src_body, pr.X, pr.trg_body, ws, _centres(pr), True, pr.mu).reshape(-1)
    out = [pinv_apply(pr, k, pr.project(k, pr.sblock(t, k)), transpose=True) for k in range(len(pr.bodies))]
    return w + np.concatenate(out)


def rhs(pr, net, rows=None):
    """b = -u_0 with s_0 from the oracle's completion (FP64 on both paths) and
    the all-pairs sum in the float32 model."""
    s0 = pr.completion_strengths(net)
    s = s0.reshape(-1, 3) if pr.kind == O.STOKES else s0
    X, tb = (pr.X, pr.trg_body) if rows is None else (pr.X[rows], pr.trg_body[rows])
    return -pair_sum(pr.kind, X, tb, pr.Y, pr.src_body, s, _centres(pr), False, pr.mu).reshape(-1)


def precond_apply(pr, v, transpose=False, project=False, qr=False):
    """The blocks as mfs_precond_apply applies them: S_L^+ v, (I - L) S_L^+ v,
    (S_L^+)^T v or (S_L^+)^T (I - L) v, per body."""
    out = []
    for k in range(len(pr.bodies)):
        if transpose:
            x = pr.sblock(v, k)
            out.append(pinv_apply(pr, k, pr.project(k, x) if project else x, transpose=True, qr=qr))
        else:
            lam = pinv_apply(pr, k, pr.gblock(v, k), qr=qr)
            out.append(pr.project(k, lam) if project else lam)
    return np.concatenate(out)


def bar(model_err: float, floor: float = 1e-15) -> float:
    """The mixed bar for a step whose float32 model errs by model_err."""
    return BAR_FACTOR * max(model_err, floor)


# GMRES stopping margin of the library (mfs_plan_set_stop_factor default)
STOP = 0.1


def solve_bars(pr, net, tol, ref=None, keys=("out",), cap=None, qr=False):
    """Bars for the outputs of a mixed solve at GMRES tol `tol`.

    Two limits, the larger of which sets the bar (times BAR_FACTOR, capped:
    1e-5 for the outputs the method reports):
    * the stopping residual: the mixed GMRES iterates until its estimate is
      at most STOP * tol; the FP64 true residual then carries the FP32
      operator's own error too (eps_mv, the float32 model's matvec error on a
      random vector), and a system above tol restarts from its iterate
      (refinement) until the true residual is at most tol.  So the solve ends
      at a residual of at most r = min(tol, max(STOP * tol, eps_mv)).  The
      oracle's GMRES stopped at r gives the ratio of output error to relative
      residual near convergence (its iterate's residual rho may lie well below
      r): this limit is that ratio x r;
    * the FP32 operator: its matvecs cannot tell the solution gamma from
      gamma + delta, delta = (A_32 - A) gamma the float32 model's matvec error
      at the solution, so the outputs are known only up to what delta does to
      them through the recovery (S_L^+ with FP64 factors, eqs. (vkal),
      (getU)): this limit is the change of each output under gamma + delta.
    ref: the oracle's solve at a tight tolerance (a dict as Problem.solve
    returns; solved here when None)."""
    if ref is None or "gamma" not in ref:
        ref = pr.solve(net, tol=1e-13)
    g = np.random.default_rng(np.random.SeedSequence(9999)).standard_normal(pr.n_gamma)
    ref_mv = pr.matvec(g)
    eps_mv = float(np.abs(matvec(pr, g, qr=qr) - ref_mv).max() / np.abs(ref_mv).max())
    r = min(tol, max(STOP * tol, eps_mv))
    sol = pr.solve(net, tol=r)
    rho = max(float(sol["hist"][-1]), 1e-300)
    gam = np.asarray(ref["gamma"])
    delta = matvec(pr, gam, qr=qr) - pr.matvec(gam)
    moved = dict(zip(("out", "lam", "sigma"), pr.extract(gam + delta, ref["s0"])))
    moved["gamma"] = gam + delta
    out = {}
    for k in keys:
        den = np.abs(np.asarray(ref[k])).max()
        err = np.abs(np.asarray(sol[k]) - np.asarray(ref[k])).max() / den
        floor = np.abs(np.asarray(moved[k]) - np.asarray(ref[k])).max() / den
        b = bar(max(err / rho * r, floor))
        out[k] = min(b, cap) if cap else b
    return out
