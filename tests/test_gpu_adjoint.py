"""Gradients of a mobility loss with respect to the particle centres and the
given net quantities: the
adjoint solve (mfs_gmres_solve_backward, the backward pair kernels, the adjoint
matvec) against the oracle's adjoint gradient and against central finite
differences of forward solves.

Loss J = sum_k |U^(k)|^2 (velocities and angular velocities), so
dJ/dU = 2 U.  Tolerances (rel_inf over the (P, 3) gradient), against the
oracle's gradient with both solves at tol 1e-14:
* FP64 plan, tol 1e-12 on both solves; MIXED plan, tol 1e-8 (FP64
  true-residual refinement on both solves): 4 x (the error of the model of
  the gradient's pair sums in the plan's precision, float64 or float32, on
  the oracle's adjoint solution and strengths + the oracle's own error when
  both its solves stop at the plan's tol), at most 1e-5
  (oracle/fp32_model.py gradient_bars); the same for dJ/d(net).
* Finite differences (h = 1e-5, FP64 solves at tol 1e-12) of the directional
  derivative along a unit direction v: |fd - g.v| <= 1e-6 |g|_2 for the FP64
  gradient and 1e-5 |g|_2 for the mixed one (the error of a directional
  derivative is measured against the gradient's norm, not against g.v, which
  can be small; truncation ~h^2, solver noise ~1e-12 J / h).
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


def _gpu_grad(wl, prec, tol):
    mfs = _mfs()
    plan = mfs.Plan.from_workload(wl, prec)
    out, info = plan.solve(_dev(net_flat(wl)), tol=tol)
    g, _, iters, relres, st = plan.gmres_solve_backward(info["gamma"], info["s0"], 2.0 * out, tol=tol)
    assert st == mfs.MFS_OK
    U = out.cpu().numpy().reshape(-1, 6)
    return float(np.sum(U * U)), g.cpu().numpy(), iters


def test_gradient_matches_oracle_small():
    mfs = _mfs()
    wl = W.small_cluster(3, W.STOKES, 60, 130, seed=31, axes=(1.0, 1.0, 1.0))
    pr = O.Problem.from_workload(wl)
    g_ref, info, b64 = M.gradient_bars(pr, wl.net[0], 1e-12, F64)
    _, _, bmx = M.gradient_bars(pr, wl.net[0], 1e-8, M.F32)
    J_ref = float(np.sum(np.asarray(info["sol"]["out"]) ** 2))
    J64, g64, _ = _gpu_grad(wl, mfs.FP64, 1e-12)
    Jmx, gmx, _ = _gpu_grad(wl, mfs.MIXED, 1e-8)
    print("J", J_ref, J64, Jmx, "grad err fp64", rel_inf(g64, g_ref), b64, "mixed", rel_inf(gmx, g_ref), bmx)
    assert abs(J64 - J_ref) <= 1e-10 * J_ref
    assert rel_inf(g64, g_ref) <= b64["centre"]
    assert rel_inf(gmx, g_ref) <= bmx["centre"]


def test_gradient_ellipsoids_matches_oracle():
    mfs = _mfs()
    wl = W.small_cluster(4, W.STOKES, 45, 301, seed=32)
    pr = O.Problem.from_workload(wl)
    g_ref, _, b64 = M.gradient_bars(pr, wl.net[0], 1e-12, F64)
    _, _, bmx = M.gradient_bars(pr, wl.net[0], 1e-8, M.F32)
    _, g64, _ = _gpu_grad(wl, mfs.FP64, 1e-12)
    _, gmx, _ = _gpu_grad(wl, mfs.MIXED, 1e-8)
    assert rel_inf(g64, g_ref) <= b64["centre"]
    assert rel_inf(gmx, g_ref) <= bmx["centre"]


def test_autograd_function():
    mfs = _mfs()
    wl = W.small_cluster(3, W.STOKES, 60, 130, seed=33, axes=(1.0, 1.0, 1.0))
    g_ref, info, bars = M.gradient_bars(O.Problem.from_workload(wl), wl.net[0], 1e-8, M.F32)
    spec = dict(precision=mfs.MIXED, sys_body_ptr=wl.sys_body_ptr, sys_kind=wl.sys_kind, rot=wl.rot,
                shape_of_body=wl.shape_of_body, shape_src=[s.src for s in wl.shapes],
                shape_trg=[s.trg for s in wl.shapes], mu=1.0, tol=1e-8)
    centre = torch.tensor(wl.centre, dtype=torch.float64, device="cuda", requires_grad=True)
    net = _dev(net_flat(wl)).requires_grad_(True)
    U = mfs.MobilitySolve.apply(centre, net, spec)
    loss = (U * U).sum()
    loss.backward()
    print("autograd: centre grad err", rel_inf(centre.grad.cpu().numpy(), g_ref),
          "net grad err", rel_inf(net.grad.cpu().numpy(), info["grad_net"].reshape(-1)))
    assert rel_inf(centre.grad.cpu().numpy(), g_ref) <= bars["centre"]
    assert rel_inf(net.grad.cpu().numpy(), info["grad_net"].reshape(-1)) <= bars["net"]


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_net_gradient_matches_oracle(kind):
    """dJ/d(net) (forces and torques, or charges) of J = sum |U|^2 or sum phi^2
    from mfs_gmres_solve_backward against the oracle's (itself pinned by
    central differences of whole solves in the net quantities), together with
    the centre gradient from the same call; NULL strength0 with a centre
    gradient requested is refused."""
    mfs = _mfs()
    wl = W.small_cluster(4, kind, 45, 301, seed=35)
    pr = O.Problem.from_workload(wl)
    for prec, tol, dt in ((mfs.FP64, 1e-12, F64), (mfs.MIXED, 1e-8, M.F32)):
        g_ref, info_ref, bars = M.gradient_bars(pr, wl.net[0], tol, dt)
        gn_ref = info_ref["grad_net"].reshape(-1)
        plan = mfs.Plan.from_workload(wl, prec)
        out, info = plan.solve(_dev(net_flat(wl)), tol=tol)
        gc, gn, iters, _, st = plan.gmres_solve_backward(info["gamma"], info["s0"], 2.0 * out, tol=tol,
                                                         want_net=True)
        assert st == mfs.MFS_OK
        e = (rel_inf(gc.cpu().numpy(), g_ref), rel_inf(gn.cpu().numpy(), gn_ref))
        print(f"kind={kind} prec={prec} centre grad err {e[0]:.2e} net grad err {e[1]:.2e} iters {iters}", bars)
        assert e[0] <= bars["centre"] and e[1] <= bars["net"]
        _, gn2, _, _, st = plan.gmres_solve_backward(info["gamma"], None, 2.0 * out, tol=tol, want_centre=False,
                                                     want_net=True)
        assert st == mfs.MFS_OK and rel_inf(gn2.cpu().numpy(), gn.cpu().numpy()) <= 1e-12
        with pytest.raises(mfs.MfsError) as err:
            plan.gmres_solve_backward(info["gamma"], None, 2.0 * out, tol=tol)
        assert err.value.status == mfs.MFS_EINVAL
        plan.close()


@pytest.mark.timeout(600)
def test_gradient_directional_fd_spheres_200():
    """Full-size workload (200 unit spheres, N=400, M=800): mixed adjoint
    gradient vs central differences of FP64 GPU solves along random directions."""
    mfs = _mfs()
    wl = W.spheres_200()
    J, g, iters = _gpu_grad(wl, mfs.MIXED, 1e-8)
    _, g64, _ = _gpu_grad(wl, mfs.FP64, 1e-10)
    print("J", J, "adjoint iters", iters, "mixed vs fp64 grad", rel_inf(g, g64))
    assert rel_inf(g, g64) <= 1e-5
    rng = np.random.default_rng(7)
    h = 1e-5
    base = wl.centre.copy()
    for _ in range(2):
        v = rng.standard_normal(base.shape)
        v /= np.linalg.norm(v)
        Js = []
        for sgn in (1.0, -1.0):
            wl.centre = base + sgn * h * v
            plan = mfs.Plan.from_workload(wl, mfs.FP64)
            out, _ = plan.solve(_dev(net_flat(wl)), tol=1e-12)
            Js.append(float((out * out).sum()))
            plan.close()
        wl.centre = base
        fd = (Js[0] - Js[1]) / (2 * h)
        ad = float(np.sum(g * v))
        ad64 = float(np.sum(g64 * v))
        print("directional fd", fd, "mixed", ad, "fp64", ad64)
        assert abs(fd - ad64) <= 1e-6 * np.linalg.norm(g64)
        assert abs(fd - ad) <= 1e-5 * np.linalg.norm(g)


def test_elastance_gradient_matches_oracle():
    """Laplace elastance: J = sum_k (phi^(k))^2, dJ/dphi = 2 phi, against the
    oracle's adjoint gradient (itself pinned by finite differences)."""
    mfs = _mfs()
    wl = W.small_cluster(4, W.LAPLACE, 45, 301, seed=34)
    pr = O.Problem.from_workload(wl)
    for prec, tol, dt in ((mfs.FP64, 1e-12, F64), (mfs.MIXED, 1e-8, M.F32)):
        g_ref, info_ref, bars = M.gradient_bars(pr, wl.net[0], tol, dt)
        J_ref = float(np.sum(np.asarray(info_ref["sol"]["out"]) ** 2))
        bar = bars["centre"]
        plan = mfs.Plan.from_workload(wl, prec)
        out, info = plan.solve(_dev(net_flat(wl)), tol=tol)
        g, _, iters, relres, st = plan.gmres_solve_backward(info["gamma"], info["s0"], 2.0 * out, tol=tol)
        assert st == mfs.MFS_OK
        J = float((out * out).sum())
        e = rel_inf(g.cpu().numpy(), g_ref)
        print("elastance", prec, "J", J, J_ref, "grad err", e, "adjoint iters", iters)
        assert abs(J - J_ref) <= 1e-6 * J_ref and e <= bar
        plan.close()


@pytest.mark.timeout(600)
def test_gradient_spheres_200_vs_stored_oracle():
    """Full size (200 unit spheres, N = 400, M = 800): dJ/dc and dJ/d[f; t] of
    J = sum |U|^2 against the oracle's, stored by tests/golden/make_golden.py
    grad_200 with both oracle solves at tol 1e-13.  FP64 plan at tol 1e-12 and
    mixed at tol 1e-8; bars 4 x (the model's error of the gradient on the
    stored sample of bodies, on the oracle's adjoint solution and strengths +
    the oracle's own error at the plan's tol, also stored), at most 1e-5."""
    import os
    mfs = _mfs()
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    path, path_m = os.path.join(golden, "spheres_200_gradient.txt"), os.path.join(golden, "spheres_200_gradient_model.txt")
    if not (os.path.exists(path) and os.path.exists(path_m)):
        pytest.skip("spheres_200 gradients not written yet (tests/golden/make_golden.py grad_200)")
    tab, mod = np.loadtxt(path), np.loadtxt(path_m)
    g_ref, n_ref = tab[:, 0:3], tab[:, 3:9]
    at_tol = {1e-12: (tab[:, 9:12], tab[:, 12:18]), 1e-8: (tab[:, 18:21], tab[:, 21:27])}
    bodies = mod[:, 0].astype(int)
    model = {mfs.MIXED: (mod[:, 1:4], mod[:, 4:10]), mfs.FP64: (mod[:, 10:13], mod[:, 13:19])}

    def rel(a, r):
        return float(np.abs(np.asarray(a) - r).max() / np.abs(r).max())

    def rel_rows(a, r):  # the sampled rows, against the largest entry over all bodies
        return float(np.abs(a - r[bodies]).max() / np.abs(r).max())
    wl = W.spheres_200()
    for prec, tol in ((mfs.FP64, 1e-12), (mfs.MIXED, 1e-8)):
        (gt, nt), (mc, mn) = at_tol[tol], model[prec]
        bar_c = min(1e-5, M.bar(rel_rows(mc, g_ref) + rel(gt, g_ref)))
        bar_n = min(1e-5, M.bar(rel_rows(mn, n_ref) + rel(nt, n_ref)))
        plan = mfs.Plan.from_workload(wl, prec)
        out, info = plan.solve(_dev(net_flat(wl)), tol=tol)
        gc, gn, iters, _, st = plan.gmres_solve_backward(info["gamma"], info["s0"], 2.0 * out, tol=tol,
                                                         want_net=True)
        assert info["status"] == mfs.MFS_OK and st == mfs.MFS_OK
        e = (rel(gc.cpu().numpy().reshape(-1, 3), g_ref), rel(gn.cpu().numpy().reshape(-1, 6), n_ref))
        print(f"spheres_200 prec={prec} tol={tol:g}: dJ/dc err {e[0]:.2e} (bar {bar_c:.2e}), "
              f"dJ/dnet err {e[1]:.2e} (bar {bar_n:.2e}), adjoint iters {iters}", flush=True)
        assert e[0] <= bar_c and e[1] <= bar_n
        plan.close()
