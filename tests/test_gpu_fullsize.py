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


@pytest.mark.slow
@pytest.mark.timeout(1200)
def test_ellipsoids_10000_sampled_rows():
    """The paper's large case (10^4 Type T ellipsoids, N = 658, M = 842, 5.5e13
    off-body pairs per matvec): right-hand side and matvec on 1000 sampled
    collocation rows, each computed by the oracle.  FP64: 1e-10 on a random
    input, 1e-12 on the right-hand side; mixed: 2e-5 on a smooth field and on
    the right-hand side (as for ellipsoids_1000)."""
    import time
    t0 = time.perf_counter()

    def step(what):
        print(f"[10^4 rows] {what} done, {time.perf_counter() - t0:.0f} s", flush=True)

    mfs = _mfs()
    wl = W.ellipsoids_10000(W.STOKES)
    pr = O.Problem.from_workload(wl)
    step("oracle set-up (one SVD)")
    rows = np.sort(np.random.default_rng(86).choice(pr.X.shape[0], 1000, replace=False))
    idx = pr._row_index(rows)
    g = W.random_vector(pr.n_gamma, 87)
    sm = W.smooth_vector(wl, 88)
    ref_g = pr.matvec(g, rows=rows)
    step("oracle matvec rows, random input")
    ref_sm = pr.matvec(sm, rows=rows)
    step("oracle matvec rows, smooth input")
    ref_b, _ = pr.rhs(wl.net[0], rows=rows)
    step("oracle right-hand side rows")
    plan = mfs.Plan.from_workload(wl, mfs.MIXED)
    step("GPU plan")
    for prec, inp, ref, tol, tol_b in ((mfs.FP64, g, ref_g, 1e-10, 1e-12), (mfs.MIXED, sm, ref_sm, 2e-5, 2e-5)):
        got = plan.matvec(_dev(inp), prec).cpu().numpy()[idx]
        b, _ = plan.rhs(_dev(net_flat(wl)), prec=prec)
        e = (rel_inf(got, ref), rel_inf(b.cpu().numpy()[idx], ref_b))
        print("ellipsoids_10000", prec, "matvec rows err", e[0], "rhs rows err", e[1], flush=True)
        assert e[0] <= tol and e[1] <= tol_b
    plan.close()


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
