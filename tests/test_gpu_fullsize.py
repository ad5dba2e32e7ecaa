"""Parity at the benchmark sizes, in the launch configuration bench.py times
(autotuned pair-sum launch shape).

* ellipsoids_100 (100 prolate spheroids, N=400, M=800): full solves against
  the oracle's stored solutions (tests/golden/, written by make_golden.py with
  the FP64 oracle at GMRES tol 1e-10).  FP64 GPU at tol 1e-10: 1e-8; mixed at
  tol 1e-7: 1e-6; mixed at tol 1e-6: 1e-5 (the bar); mixed at the benchmark
  tolerance 1e-5 is reported.
* ellipsoids_10000 (the paper's 10^4 Type T case): right-hand side and matvec on
  1000 sampled rows (see the test).
* ellipsoids_1000 (1000 spheroids): right-hand side and matvec on 2000
  sampled collocation rows, each row computed by the oracle from the same
  seeded inputs; and on the mixed solve, the exact net force and torque of
  the strengths (K_N^T sigma = F, eq. (force_syst)).
  Matvec tolerances: FP64 1e-10 on a random input.  Mixed: 2e-5 on a smooth
  seeded field (the kind of surface data GMRES works with; FP32 pair sums
  and FP32 pseudo-inverse blocks on smooth data), and 1e-3 on a random
  vector, whose rough part the FP32 pseudo-inverse amplifies by up to
  u32 * cond(S_L) (cond = 3.8e6 for this shape) before the smooth off-body
  kernels damp it again (measured 1.6e-4).
"""
import os

import numpy as np
import pytest
import torch

import mfs_workloads as W
from oracle import mfs_oracle as O
from tests._helpers import net_flat, rel_inf

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MIX_MATVEC_SMOOTH = 2e-5
MIX_RHS = 2e-5


def _mfs():
    from paper_2409_04215_amd import mfs
    return mfs


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).reshape(-1), dtype=torch.float64, device="cuda")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind,fname", [(W.STOKES, "ellipsoids_100_stokes_U.txt"),
                                        (W.LAPLACE, "ellipsoids_100_laplace_phi.txt")])
def test_ellipsoids_100_solve_vs_stored_oracle(kind, fname):
    mfs = _mfs()
    wl = W.ellipsoids_100(kind)
    ref = np.loadtxt(os.path.join(GOLDEN, fname)).reshape(-1)
    net = _dev(net_flat(wl))
    for prec, tol, bar in ((mfs.FP64, 1e-10, 1e-8), (mfs.MIXED, 1e-7, 1e-6), (mfs.MIXED, 1e-6, 1e-5),
                           (mfs.MIXED, 1e-5, None)):
        plan = mfs.Plan.from_workload(wl, prec)
        plan.autotune(prec, reps=1)
        out, info = plan.solve(net, tol=tol)
        e = rel_inf(out.cpu().numpy(), ref)
        print(f"kind={kind} prec={prec} tol={tol:g} iters={info['iters']} relres={info['relres']} err={e:.2e}")
        assert info["status"] == mfs.MFS_OK
        if bar is not None:
            assert e <= bar
        plan.close()


_BIG = {}


def _big(kind):
    if kind not in _BIG:
        wl = W.ellipsoids_1000(kind)
        pr = O.Problem.from_workload(wl)
        rows = np.sort(np.random.default_rng(81).choice(pr.X.shape[0], 2000, replace=False))
        _BIG[kind] = (wl, pr, rows)
    return _BIG[kind]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_ellipsoids_1000_sampled_rows(kind):
    mfs = _mfs()
    wl, pr, rows = _big(kind)
    idx = pr._row_index(rows)
    g = W.random_vector(pr.n_gamma, 82)
    sm = W.smooth_vector(wl, 83)
    ref_mv = pr.matvec(g, rows=rows)
    ref_sm = pr.matvec(sm, rows=rows)
    ref_b, _ = pr.rhs(wl.net[0], rows=rows)
    plan = mfs.Plan.from_workload(wl, mfs.MIXED)
    plan.autotune(mfs.MIXED, reps=1)
    for prec, tol_rand, tol_sm, tol_b in ((mfs.FP64, 1e-10, 1e-10, 1e-12), (mfs.MIXED, 1e-3, 2e-5, 2e-5)):
        got = plan.matvec(_dev(g), prec).cpu().numpy()[idx]
        got_sm = plan.matvec(_dev(sm), prec).cpu().numpy()[idx]
        b, _ = plan.rhs(_dev(net_flat(wl)), prec=prec)
        e = (rel_inf(got, ref_mv), rel_inf(got_sm, ref_sm), rel_inf(b.cpu().numpy()[idx], ref_b))
        print(kind, prec, "matvec rows err (random, smooth)", e[0], e[1], "rhs rows err", e[2])
        assert e[0] <= tol_rand and e[1] <= tol_sm and e[2] <= tol_b


@pytest.mark.timeout(900)
def test_ellipsoids_1000_solve_invariants():
    mfs = _mfs()
    wl, pr, _ = _big(W.STOKES)
    plan = mfs.Plan.from_workload(wl, mfs.MIXED)
    plan.autotune(mfs.MIXED, reps=1)
    out, info = plan.solve(_dev(net_flat(wl)), tol=1e-5)
    assert info["status"] == mfs.MFS_OK and info["relres"][0] <= 1e-5
    _, sigma = plan.extract(info["gamma"], info["s0"], want_sigma=True)
    sigma = sigma.cpu().numpy()
    F = wl.net[0]
    worst = 0.0
    for k, b in enumerate(pr.bodies):
        FK = O.K_matrix(b.Y, b.centre).T @ pr.sblock(sigma, k)
        worst = max(worst, np.abs(FK - F[k]).max() / np.abs(F).max())
    print("iters", info["iters"], "relres", info["relres"], "net force/torque mismatch", worst)
    assert worst <= 1e-12


_E4 = {}


def _e4():
    """The 10^4 case, its stored oracle rows and one resident plan shared by the
    tests below (one SVD of the Type T block, pair records for 6.58e6 proxies)."""
    if not _E4:
        mfs = _mfs()
        tab = np.loadtxt(os.path.join(GOLDEN, "ellipsoids_10000_rows.txt"))
        wl = W.ellipsoids_10000(W.STOKES)
        plan = mfs.Plan.from_workload(wl, mfs.MIXED)
        rows = tab[:, 0].astype(np.int64)
        idx = (3 * rows[:, None] + np.arange(3)[None, :]).reshape(-1)
        _E4.update(wl=wl, plan=plan, idx=idx, b=tab[:, 1:4].reshape(-1), Ag=tab[:, 4:7].reshape(-1),
                   As=tab[:, 7:10].reshape(-1))
    return _E4


@pytest.mark.timeout(600)
def test_ellipsoids_10000_fp64_matvec_rows():
    """The paper's large case (Section 4.2: 10^4 Type T ellipsoids, N = 658,
    M = 842, 5.5e13 off-body pairs per matvec): the FP64 matvec of a seeded
    random vector on 1000 collocation rows against the oracle's rows stored
    by tests/golden/make_golden.py rows_10000 (each row summed over all
    6.58e6 proxies).  Bar 1e-10: FP64 pair sums and FP64 factors (measured
    7.5e-12)."""
    mfs = _mfs()
    e = _e4()
    g = W.random_vector(e["plan"].n_gamma, 87)
    got = e["plan"].matvec(_dev(g), mfs.FP64).cpu().numpy()[e["idx"]]
    err = rel_inf(got, e["Ag"])
    print(f"ellipsoids_10000 FP64 matvec rows err {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.timeout(600)
def test_ellipsoids_10000_mixed_rows():
    """The same case in mixed precision: the right-hand side (pair sum over all
    pairs, self included) and the matvec of a seeded smooth field on the
    stored oracle rows."""
    mfs = _mfs()
    e = _e4()
    sm = W.smooth_vector(e["wl"], 88)
    got = e["plan"].matvec(_dev(sm), mfs.MIXED).cpu().numpy()[e["idx"]]
    b, _ = e["plan"].rhs(_dev(net_flat(e["wl"])), prec=mfs.MIXED)
    err = (rel_inf(got, e["As"]), rel_inf(b.cpu().numpy()[e["idx"]], e["b"]))
    print(f"ellipsoids_10000 mixed matvec rows err {err[0]:.2e}, rhs rows err {err[1]:.2e}", flush=True)
    assert err[0] <= MIX_MATVEC_SMOOTH and err[1] <= MIX_RHS
    e["plan"].close()
    _E4.clear()


@pytest.mark.timeout(600)
def test_ellipsoids_100_two_way_vs_stored_oracle():
    """The 2-way test (eq. (2way)) at the benchmark size: resistance solve with
    the stored rigid velocities U_ref (proxies at the resistance scale), then
    the mobility solve with the resulting forces (proxies at 0.7); F, U and
    eps_2way against the oracle's stored run (tests/golden/, FP64 at tol
    1e-10).  FP64 at tol 1e-10: F and U within 1e-8; mixed at tol 1e-6:
    within 1e-5; eps_2way within the same bound (it is a difference of U)."""
    mfs = _mfs()
    tab = np.loadtxt(os.path.join(GOLDEN, "ellipsoids_100_two_way.txt"))
    U_ref, F_ref, U_2 = tab[:, :6], tab[:, 6:12], tab[:, 12:]
    eps_ref = np.abs(U_2 - U_ref).max() / np.abs(U_ref).max()
    wl = W.ellipsoids_100(W.STOKES)
    wr = W.with_proxy_scale(wl, W.resistance_proxy_scale())
    for prec, tol, bar in ((mfs.FP64, 1e-10, 1e-8), (mfs.MIXED, 1e-6, 1e-5)):
        res = mfs.Plan.from_workload(wr, prec, formulation=mfs.RESISTANCE)
        mob = mfs.Plan.from_workload(wl, prec)
        F, ir = res.solve(_dev(U_ref), tol=tol)
        U, im = mob.solve(F, tol=tol)
        F, U = F.cpu().numpy(), U.cpu().numpy()
        eps = np.abs(U - U_ref.reshape(-1)).max() / np.abs(U_ref).max()
        e = (rel_inf(F, F_ref), rel_inf(U, U_2), abs(eps - eps_ref))
        print(f"prec={prec} tol={tol:g} iters res {ir['iters']} mob {im['iters']} F err {e[0]:.2e} "
              f"U err {e[1]:.2e} eps_2way {eps:.4e} (oracle {eps_ref:.4e})", flush=True)
        assert ir["status"] == mfs.MFS_OK and im["status"] == mfs.MFS_OK
        assert max(e) <= bar
        res.close()
        mob.close()
