"""Checks of the arithmetic models that size the parity bars
(oracle/fp32_model.py), on the CPU: each model must err the way it claims to.

* float64 model of a factorisation: the exact SVD of S_L + E with
  |E|_2 = u64 |S_L|_2, so its backward error is that of LAPACK's own SVD, and
  its pseudo-inverse differs from the oracle's by about u64 cond(S_L), as an
  independently rounded FP64 factorisation does.
* float32 model of a pair sum: its error against the FP64 oracle lies between
  the unit roundoff and the worst-case bound u32 x (run length + runs) x
  sum |terms| / max |u|, i.e. it is rounding error of float32 size.
* float64 model of a pair sum: the same with u64.
* the mixed QR plan's model keeps R^-1 in FP64: its pseudo-inverse error is of
  float32 size, not that of an FP32 R^-1.
"""
import numpy as np

import mfs_workloads as W
from oracle import fp32_model as M
from oracle import mfs_oracle as O

U64 = np.finfo(np.float64).eps / 2
U32 = float(np.finfo(np.float32).eps) / 2


def _problem(kind, seed=301):
    return O.Problem.from_workload(W.small_cluster(3, kind, 30, 90, seed=seed))


def test_float64_factor_model_is_an_independent_backward_stable_factorisation():
    """Its backward error is that of LAPACK's own SVD (within 2x of the oracle's
    factors), and its pseudo-inverse differs from the oracle's by an amount of
    the order of u64 cond(S_L) (not the far smaller difference of two SVDs that
    share their rounding), at most 4 u64 cond(S_L)."""
    L = np.longdouble
    for kind in (W.STOKES, W.LAPLACE):
        pr = _problem(kind)
        key = next(iter(pr.factors))
        F = pr.factors[key]
        Ut, Wm, U, Wt = M._factors(pr, F, key, False, np.float64)
        S = M._block_matrix(pr, key).astype(L)
        sigma = 1.0 / np.sqrt((Wm.astype(L) ** 2).sum(axis=0))
        back_model = float(np.abs(S - (U.astype(L) * sigma) @ (Wm.astype(L) * sigma).T).max() / np.abs(S).max())
        back_oracle = float(np.abs(S - (F.U.astype(L) * F.s.astype(L)) @ F.Vt.astype(L)).max() / np.abs(S).max())
        assert back_model <= 2 * back_oracle + 2 * U64, (back_model, back_oracle)
        g = W.random_vector(S.shape[0], 302)
        ref = F.apply(g)
        err = np.abs(Wm @ (Ut @ g) - ref).max() / np.abs(ref).max()
        cond = 1.0 / F.ratio
        assert 0.002 * U64 * cond <= err <= 4 * U64 * cond, (err, cond)


def _terms_scale(kind, X, tb, Y, sb, s):
    """A bound of sum_j |G(x_i - y_j) s_j| per target (off-body pairs): the
    Laplace kernel 1/(4 pi r) on |s|; a Stokeslet term is at most
    (|s| + |d| |d.s| / r^2) / (8 pi r) <= |s| / (4 pi r)."""
    mag = np.abs(s) if kind == W.LAPLACE else np.linalg.norm(s, axis=1)
    return O.p2p(W.LAPLACE, X, tb, Y, sb, mag, 1.0, True)


def test_pair_sum_models_err_at_their_precision():
    for kind in (W.STOKES, W.LAPLACE):
        wl = W.small_cluster(3, kind, 40, 200, seed=303)
        X, tb = wl.world_points("trg")
        Y, sb = wl.world_points("src")
        s = np.random.default_rng(304).standard_normal((Y.shape[0], 3) if kind == W.STOKES else Y.shape[0])
        ref = O.p2p(kind, X, tb, Y, sb, s, 1.0, True)
        first = M.ref_first_source(wl.n_body, sb, Y, tb, X)
        scale = np.abs(_terms_scale(kind, X, tb, Y, sb, s)).max() / np.abs(ref).max()
        n_src = Y.shape[0]
        for dt, u in ((M.F32, U32), (np.float64, U64)):
            err = np.abs(M.pair_sum(kind, X, tb, Y, sb, s, first, dt=dt) - ref).max() / np.abs(ref).max()
            bound = u * (M.RUN + n_src / M.RUN + 20) * max(scale, 1.0)
            assert 0.1 * u <= err <= bound, (kind, dt, err, bound)


def test_mixed_qr_model_keeps_the_triangular_factor_in_fp64():
    pr = _problem(W.STOKES, seed=305)
    key = next(iter(pr.factors))
    Qt, Ri, Q, RiT = M._factors(pr, pr.factors[key], key, True, M.F32)
    assert Qt.dtype == np.float32 and Q.dtype == np.float32
    assert Ri.dtype == np.float64 and RiT.dtype == np.float64
    g = W.random_vector(pr.n_gamma, 306)
    ref = np.concatenate([pr.pinv_apply(k, pr.gblock(g, k)) for k in range(len(pr.bodies))])
    err = np.abs(M.precondition(pr, g, project=False, qr=True) - ref).max() / np.abs(ref).max()
    F = pr.factors[key]
    assert err <= 64 * U32 / F.ratio, err
