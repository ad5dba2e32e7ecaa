"""The paper's small elastance test (Section 4.1) at its own sizes on the GPU:
10 unit spheres grown compactly at delta = 0.1, R_p = 0.7, N = 969, M = 1123,
GMRES tolerance 1e-8 (values in tests/golden/paper_elastance_spheres.txt).

The oracle's GMRES at tol needs 15 iterations, the paper's count.  The plans
here use the paper's stopping rule as stated (mfs_plan_set_stop_factor(1):
stop once the residual estimate is below tol), so the GPU is compared with
the oracle run to tol:
* FP64 plan: the paper's and the oracle's iteration count, the same maximum
  surface residual |u - phi| (4000 points per sphere) to 1e-3 of itself.
* Mixed plan at the same tolerance (FP64 true-residual refinement): surface
  residual within 1e-2 of the oracle's maximum.
* Both: potentials against the oracle's tight solution (tol 1e-12) within
  4 x the larger of the stopping limit and the operator limit
  (oracle/fp32_model.py solve_bars with the model of the plan's precision
  and the stopping factor 1 these plans use),
  and the GPU solution's residual under the oracle's b and A at most tol
  plus 4 x the model's right-hand-side error.
"""
import os

import numpy as np
import pytest
import torch

import mfs_workloads as W
from oracle import mfs_oracle as O
from oracle import fp32_model as M
from tests._helpers import rel_inf

pytestmark = pytest.mark.gpu


def _mfs():
    from paper_2409_04215_amd import mfs
    return mfs


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).reshape(-1), dtype=torch.float64, device="cuda")


def _ref():
    vals = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_elastance_spheres.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


@pytest.mark.timeout(300)
def test_paper_elastance_example_on_gpu():
    mfs = _mfs()
    ref = _ref()
    wl = W.elastance_spheres(int(ref["N"]), int(ref["M"]), n_body=int(ref["P"]), delta=ref["delta"])
    tol = ref["gmres_tol"]
    pr = O.Problem.from_workload(wl)
    assert abs(pr.solve(wl.net[0], tol=tol)["iters"] - ref["gmres_iterations"]) <= 1
    sol = pr.solve(wl.net[0], tol=tol)
    tight = pr.solve(wl.net[0], tol=1e-12)
    test = W.fibonacci_sphere(4000, 1.0)
    eps_ref = pr.surface_residual(sol["sigma"], sol["out"], test).max()
    for prec, dt, eps_bar in ((mfs.FP64, np.float64, 1e-3), (mfs.MIXED, M.F32, 1e-2)):
        plan = mfs.Plan.from_workload(wl, prec)
        plan.set_stop_factor(1.0)
        out, info = plan.solve(_dev(wl.net[0]), tol=tol)
        _, sigma = plan.extract(info["gamma"], info["s0"], want_sigma=True)
        eps = plan.surface_residual(sigma, out, test).cpu().numpy().max()
        e = rel_inf(out.cpu().numpy(), tight["out"])
        bars = M.solve_bars(pr, wl.net[0], tol, tight, dt=dt, gamma=info["gamma"].cpu().numpy(), stop=1.0)
        print("paper elastance", prec, "iters", info["iters"], "oracle iters", sol["iters"], "phi err", e, bars,
              "max |u - phi|", eps, "oracle", eps_ref)
        assert info["status"] == mfs.MFS_OK and bars["residual"] <= bars["residual_bound"] and e <= bars["out"]
        assert abs(eps - eps_ref) <= eps_bar * eps_ref
        if prec == mfs.FP64:
            assert info["iters"][0] == sol["iters"]
        plan.close()


@pytest.mark.parametrize("delta", [0.2, 0.5])
def test_two_spheres_exact_on_gpu(delta):
    """Two unit spheres, equal forces along the line of centres (the paper's
    two-sphere comparison setting, Appendix A.1): GPU velocities against the exact
    Stimson-Jeffery solution.  N = 800, M = 1600: FP64 within 1e-8 (the MFS
    discretisation error here is 4e-10), mixed at tol 1e-7 within 1e-6."""
    from tests._helpers import stimson_jeffery_lambda, two_sphere_workload
    mfs = _mfs()
    exact = 1.0 / (6.0 * np.pi * stimson_jeffery_lambda(2.0 + delta))
    wl = two_sphere_workload(W, delta, 800, 1600)
    for prec, tol, bar in ((mfs.FP64, 1e-12, 1e-8), (mfs.MIXED, 1e-7, 1e-6)):
        plan = mfs.Plan.from_workload(wl, prec)
        out, info = plan.solve(_dev(wl.net[0]), tol=tol)
        U = out.cpu().numpy().reshape(2, 6)
        err = np.abs(U[:, 0] - exact).max() / exact
        print("two spheres", delta, prec, "U_x", U[:, 0], "exact", exact, "rel err", err)
        assert info["status"] == mfs.MFS_OK and err <= bar
        plan.close()
