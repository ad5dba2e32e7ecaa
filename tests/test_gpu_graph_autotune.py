"""hipGraph replay of the GMRES matvec and the launch-shape autotuner.

* Graph: solves with the captured matvec, replayed many times inside GMRES,
  repeated with eager work and synchronisations in between, must equal the
  eager solve bit for bit (the same kernels in the same order on the same
  data; only the Krylov column is staged into a fixed buffer first).
* Autotune: after the pair-sum launch shape changes, the matvec still agrees
  with the oracle (the bars of test_gpu_operator: 4 x the error of the
  model of each precision) and solves converge.
"""
import numpy as np
import pytest
import torch

import mfs_workloads as W
from oracle import mfs_oracle as O
from oracle import fp32_model as M
from tests._helpers import net_flat, rel_inf

pytestmark = pytest.mark.gpu

F64 = np.float64


def _mfs():
    from paper_2409_04215_amd import mfs
    return mfs


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).reshape(-1), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_graph_replay_equals_eager(kind):
    mfs = _mfs()
    wl = W.small_cluster(5, kind, 45, 301, seed=71)
    net = _dev(net_flat(wl))
    for prec in (mfs.MIXED, mfs.FP64):
        plan = mfs.Plan.from_workload(wl, prec)
        eager, info_e = plan.solve(net, tol=1e-9)
        plan.set_graph(True)
        g = _dev(W.random_vector(plan.n_gamma, 72))
        for rep in range(3):
            out, info = plan.solve(net, tol=1e-9)
            torch.cuda.synchronize()
            assert torch.equal(out, eager), (prec, rep)
            assert np.array_equal(info["iters"], info_e["iters"])
            # eager work between replays
            plan.matvec(g, prec)
            torch.cuda.synchronize()
        # the adjoint solve replays its own graph
        b, _ = plan.rhs(net)
        plan.set_graph(False)
        ge, *_ = plan.gmres_solve(b, tol=1e-9, adjoint=True)
        plan.set_graph(True)
        for rep in range(2):
            gg, *_ = plan.gmres_solve(b, tol=1e-9, adjoint=True)
            torch.cuda.synchronize()
            assert torch.equal(gg, ge)
        plan.close()


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_autotune_keeps_results(kind):
    mfs = _mfs()
    wl = W.small_cluster(5, kind, 45, 301, seed=73)
    pr = O.Problem.from_workload(wl)
    g = W.random_vector(pr.n_gamma, 74)
    ref = pr.matvec(g)
    plan = mfs.Plan.from_workload(wl, mfs.MIXED)
    tpl, mi, ms = plan.autotune(mfs.MIXED, reps=2)
    assert abs(tpl) in (1, 2) and mi in (1024, 2048, 4096, 8192, 16384) and ms > 0
    ref_t = pr.matvec_T(g)
    assert rel_inf(plan.matvec(_dev(g), mfs.FP64).cpu().numpy(), ref) <= M.bar(rel_inf(M.matvec(pr, g, dt=F64), ref))
    assert rel_inf(plan.matvec(_dev(g), mfs.MIXED).cpu().numpy(), ref) <= M.bar(rel_inf(M.matvec(pr, g), ref))
    assert rel_inf(plan.matvec_adjoint(_dev(g), mfs.FP64).cpu().numpy(), ref_t) <= \
        M.bar(rel_inf(M.matvec_T(pr, g, dt=F64), ref_t))
    out, info = plan.solve(_dev(net_flat(wl)), tol=1e-8)
    assert info["status"] == mfs.MFS_OK
    sol = pr.solve(wl.net[0], tol=1e-12)
    bars = M.solve_bars(pr, wl.net[0], 1e-8, sol, cap=1e-5, gamma=info["gamma"].cpu().numpy())
    assert bars["residual"] <= bars["residual_bound"]
    assert rel_inf(out.cpu().numpy(), sol["out"]) <= bars["out"]


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_every_launch_shape(kind):
    """Each launch shape the autotuner can pick (targets per lane, work items,
    persistent work-queue grid) gives the same operator."""
    mfs = _mfs()
    wl = W.small_cluster(6, kind, 45, 301, seed=75)
    pr = O.Problem.from_workload(wl)
    g = W.random_vector(pr.n_gamma, 76)
    ref, ref_t = pr.matvec(g), pr.matvec_T(g)

    def bar(dt):
        return M.bar(max(rel_inf(M.matvec(pr, g, dt=dt), ref), rel_inf(M.matvec_T(pr, g, dt=dt), ref_t)))
    bars = {mfs.FP64: bar(F64), mfs.MIXED: bar(M.F32)}
    plan = mfs.Plan.from_workload(wl, mfs.MIXED)
    for tpl in (1, 2):
        for items in (1, 64, 16384):
            for per in (False, True):
                plan.set_launch(tpl, items, per)
                for prec, tol in bars.items():
                    e = (rel_inf(plan.matvec(_dev(g), prec).cpu().numpy(), ref),
                         rel_inf(plan.matvec_adjoint(_dev(g), prec).cpu().numpy(), ref_t))
                    assert max(e) <= tol, (tpl, items, per, prec, e)
    # a persistent-grid solve replayed from a graph equals the eager one
    plan.set_launch(1, 16384, True)
    net = _dev(net_flat(wl))
    eager, _ = plan.solve(net, tol=1e-9)
    plan.set_graph(True)
    for _ in range(2):
        out, _ = plan.solve(net, tol=1e-9)
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
