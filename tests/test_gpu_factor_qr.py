"""The library's batched FP64 Householder QR as the one-body factorisation
(MFS_FACTOR_QR): S_L = Q R, S_L^+ = R^-1 Q^T, applied as (R^-1)(Q^T .).

For full column rank this is the pseudo-inverse the SVD gives (Section 2.3),
so a QR plan must meet the same bars against the oracle (which uses the SVD)
as an SVD plan, and agree with an SVD plan to FP64 rounding amplified by the
conditioning of S_L:
* S_L^+ apply and Ag: 4 x the error of the model with a QR plan's factors
  Q^T and R^-1 (oracle/fp32_model.py: float32 factors and products for
  mixed; an independent FP64 QR and R^-1 for FP64);
* solves: at tol t within 4 x the larger of the stopping limit and the
  operator limit of oracle/fp32_model.py solve_bars (QR model of the plan's
  precision), at most 1e-5, and the GPU solution's residual under the
  oracle's b and A at most t plus 4 x the model's right-hand-side error;
  ellipsoids_100 against the stored oracle solutions as in the full-size
  tests;
* the reported ratio 1/(|R|_F |R^-1|_F) lies between sigma_min/sigma_max / n
  and sigma_min/sigma_max (n = columns);
* a rank-deficient block (two proxies at one point) is refused.
"""
import os
import time

import numpy as np
import pytest
import torch

import mfs_workloads as W
from oracle import mfs_oracle as O
from oracle import fp32_model as M
from tests._helpers import net_flat, rel_inf, tight_reference

pytestmark = pytest.mark.gpu
F64 = np.float64
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _mfs():
    from paper_2409_04215_amd import mfs
    return mfs


def _dev(x):
    return torch.tensor(np.ascontiguousarray(x, dtype=np.float64).reshape(-1), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_qr_plan_matches_oracle_and_svd_plan(kind):
    mfs = _mfs()
    wl = W.small_cluster(5, kind, 45, 301, seed=161)
    pr = O.Problem.from_workload(wl)
    g = W.random_vector(pr.n_gamma, 162)
    ref_p = np.concatenate([pr.pinv_apply(k, pr.gblock(g, k)) for k in range(wl.n_body)])
    ref_A = pr.matvec(g)
    sol = pr.solve(wl.net[0], tol=1e-12)
    svd = mfs.Plan.from_workload(wl, mfs.FP64)
    for prec, dt, solve_tol in ((mfs.FP64, F64, 1e-10), (mfs.MIXED, M.F32, 1e-7)):
        tol_p = M.bar(rel_inf(M.precond_apply(pr, g, qr=True, dt=dt), ref_p))
        tol_A = M.bar(rel_inf(M.matvec(pr, g, qr=True, dt=dt), ref_A))
        qr = mfs.Plan.from_workload(wl, prec, factorization=mfs.FACTOR_QR)
        e = (rel_inf(qr.precond_apply(_dev(g), 0, prec).cpu().numpy(), ref_p),
             rel_inf(qr.matvec(_dev(g), prec).cpu().numpy(), ref_A))
        out, info = qr.solve(_dev(net_flat(wl)), tol=solve_tol)
        es = rel_inf(out.cpu().numpy(), sol["out"])
        print(kind, prec, "S_L^+ apply, A g", e, "solve", es, "iters", info["iters"], "ratio bound", qr.min_sigma_ratio,
              "svd ratio", svd.min_sigma_ratio)
        assert e[0] <= tol_p and e[1] <= tol_A
        assert info["status"] == mfs.MFS_OK
        bars = M.solve_bars(pr, wl.net[0], solve_tol, sol, cap=1e-5, qr=True, dt=dt, gamma=info["gamma"].cpu().numpy())
        assert bars["residual"] <= bars["residual_bound"] and es <= bars["out"]
        if prec == mfs.FP64:
            # two FP64 factorisations of S_L: each matvec within its own bar of the oracle's
            d = rel_inf(qr.matvec(_dev(g), mfs.FP64).cpu().numpy(), svd.matvec(_dev(g), mfs.FP64).cpu().numpy())
            assert d <= tol_A + M.bar(rel_inf(M.matvec(pr, g, dt=F64), ref_A))
            ncol = (3 if kind == W.STOKES else 1) * wl.shapes[0].src.shape[0]
            assert svd.min_sigma_ratio / ncol <= qr.min_sigma_ratio <= svd.min_sigma_ratio * (1 + 1e-9)
        qr.close()
    svd.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind,fname", [(W.STOKES, "ellipsoids_100_stokes_U_tight.txt"),
                                        (W.LAPLACE, "ellipsoids_100_laplace_phi_tight.txt")])
def test_qr_plan_ellipsoids_100_vs_stored_oracle(kind, fname):
    """Against the oracle's solution at tol 1e-13, with the bars of the SVD
    plan's test (tests/test_gpu_fullsize.py)."""
    mfs = _mfs()
    wl = W.ellipsoids_100(kind)
    ref, rho, err10 = tight_reference(os.path.join(GOLDEN, fname))
    net = _dev(net_flat(wl))
    for prec, tol, bar in ((mfs.FP64, 1e-10, M.bar(err10 / rho * M.STOP * 1e-10)), (mfs.MIXED, 1e-5, 1e-5)):
        plan = mfs.Plan.from_workload(wl, prec, factorization=mfs.FACTOR_QR)
        out, info = plan.solve(net, tol=tol)
        e = rel_inf(out.cpu().numpy(), ref)
        print(f"QR kind={kind} prec={prec} tol={tol:g} iters={info['iters']} err={e:.2e} bar={bar:.2e}")
        assert info["status"] == mfs.MFS_OK and e <= bar
        plan.close()


@pytest.mark.parametrize("fact", ["FACTOR_SVD", "FACTOR_QR"])
def test_rank_deficient_block_is_refused(fact):
    mfs = _mfs()
    wl = W.small_cluster(2, W.LAPLACE, 40, 100, seed=163)
    src = wl.shapes[0].src.copy()
    src[7] = src[3]  # two proxies at one point: two equal columns of S_L
    wl.shapes[0].src = src
    with pytest.raises(mfs.MfsError) as err:
        mfs.Plan.from_workload(wl, mfs.FP64, factorization=getattr(mfs, fact))
    assert err.value.status == mfs.MFS_ENUMERIC


@pytest.mark.timeout(600)
def test_type_t_cluster_both_factorizations(capsys):
    """20 Type T ellipsoids built like the 10^4 case (N = 658, M = 842: blocks of
    2526 x 1974): solves of SVD and QR plans against the oracle.  Minutes of
    oracle work on the host: each step reports as it ends, past output capture."""
    mfs = _mfs()
    wl = W.type_t_cluster(20, W.STOKES, 164)
    pr = O.Problem.from_workload(wl)
    sol = pr.solve(wl.net[0], tol=1e-12)
    with capsys.disabled():
        print(f"\ntype T: oracle solve done ({sol['iters']} iterations)", flush=True)
    ref = sol["out"]
    net = _dev(net_flat(wl))
    for fact in (mfs.FACTOR_SVD, mfs.FACTOR_QR):
        for prec, tol, dt in ((mfs.FP64, 1e-10, F64), (mfs.MIXED, 1e-6, M.F32)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan = mfs.Plan.from_workload(wl, prec, factorization=fact)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            out, info = plan.solve(net, tol=tol)
            e = rel_inf(out.cpu().numpy(), ref)
            bars = M.solve_bars(pr, wl.net[0], tol, sol, cap=1e-5, qr=fact == mfs.FACTOR_QR, dt=dt,
                                gamma=info["gamma"].cpu().numpy())
            with capsys.disabled():
                print("type T", "QR" if fact else "SVD", prec, "iters", info["iters"], "err", e, bars,
                      "ratio", plan.min_sigma_ratio, f"plan creation {t_setup:.3f} s", flush=True)
            assert info["status"] == mfs.MFS_OK and bars["residual"] <= bars["residual_bound"] and e <= bars["out"]
            plan.close()


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_qr_resistance_plan(kind):
    """The Dirichlet formulation factors the bare S^(kk) blocks (eq. (2sysprec)); QR there too."""
    mfs = _mfs()
    wl = W.small_cluster(4, kind, 45, 301, seed=165)
    rng = np.random.default_rng(166)
    data = rng.standard_normal((4, 6)) if kind == W.STOKES else rng.standard_normal(4)
    rp = O.ResistanceProblem.from_workload(wl)
    sol = rp.solve(data, tol=1e-12)
    for prec, tol, dt in ((mfs.FP64, 1e-10, F64), (mfs.MIXED, 1e-7, M.F32)):
        plan = mfs.Plan.from_workload(wl, prec, formulation=mfs.RESISTANCE, factorization=mfs.FACTOR_QR)
        out, info = plan.solve(_dev(data), tol=tol)
        e = rel_inf(out.cpu().numpy(), np.asarray(sol["out"]).reshape(-1))
        bars = M.solve_bars(rp, data, tol, sol, cap=1e-5, qr=True, dt=dt, gamma=info["gamma"].cpu().numpy())
        print("resistance QR", kind, prec, "err", e, bars)
        assert info["status"] == mfs.MFS_OK and bars["residual"] <= bars["residual_bound"] and e <= bars["out"]
        plan.close()


@pytest.mark.parametrize("kind,n_src,n_trg", [(W.LAPLACE, 10, 30), (W.STOKES, 10, 10), (W.STOKES, 11, 40),
                                              (W.LAPLACE, 64, 64)])
def test_qr_small_square_and_ragged_blocks(kind, n_src, n_trg):
    """Blocks narrower than one 16-column panel (10 columns), a whole panel and a
    ragged one (30 = 16 + 14), square blocks (M = N: S_L^+ is the inverse; 64 =
    4 x 16 columns), and a width one column past whole panels (33 = 2 x 16 + 1):
    pseudo-inverse apply and matvec of QR plans against the oracle, within 4 x
    the model of a QR plan of the same precision."""
    mfs = _mfs()
    wl = W.small_cluster(3, kind, n_src, n_trg, seed=167, axes=(1.0, 1.0, 1.5))
    pr = O.Problem.from_workload(wl)
    g = W.random_vector(pr.n_gamma, 168)
    ref_p = np.concatenate([pr.pinv_apply(k, pr.gblock(g, k)) for k in range(wl.n_body)])
    ref_A = pr.matvec(g)
    for prec, dt in ((mfs.FP64, F64), (mfs.MIXED, M.F32)):
        plan = mfs.Plan.from_workload(wl, prec, factorization=mfs.FACTOR_QR)
        e = (rel_inf(plan.precond_apply(_dev(g), 0, prec).cpu().numpy(), ref_p),
             rel_inf(plan.matvec(_dev(g), prec).cpu().numpy(), ref_A))
        bars = (M.bar(rel_inf(M.precond_apply(pr, g, qr=True, dt=dt), ref_p)),
                M.bar(rel_inf(M.matvec(pr, g, qr=True, dt=dt), ref_A)))
        print("QR", kind, n_src, n_trg, prec, "errors", e, "bars", bars)
        assert e[0] <= bars[0] and e[1] <= bars[1]
        plan.close()


@pytest.mark.parametrize("kind", [W.STOKES, W.LAPLACE])
def test_qr_adjoint_matvec_and_transpose_blocks(kind):
    """The transposed blocks of a QR plan ((S_L^+)^T = Q R^-T: R^-T in FP64, then Q
    in FP32 for mixed plans) in the adjoint matvec and in precond_apply, against
    the oracle within 4 x the QR model of each precision."""
    mfs = _mfs()
    wl = W.small_cluster(4, kind, 45, 301, seed=169)
    pr = O.Problem.from_workload(wl)
    w = W.random_vector(pr.n_gamma, 170)
    v = W.random_vector(pr.n_lambda, 171)
    ref_t = pr.matvec_T(w)
    ref_p = np.concatenate([pr.pinv_apply_T(k, pr.sblock(v, k)) for k in range(wl.n_body)])
    for prec, dt in ((mfs.FP64, F64), (mfs.MIXED, M.F32)):
        plan = mfs.Plan.from_workload(wl, prec, factorization=mfs.FACTOR_QR)
        e = (rel_inf(plan.matvec_adjoint(_dev(w), prec).cpu().numpy(), ref_t),
             rel_inf(plan.precond_apply(_dev(v), mfs.TRANSPOSE, prec).cpu().numpy(), ref_p))
        bars = (M.bar(rel_inf(M.matvec_T(pr, w, qr=True, dt=dt), ref_t)),
                M.bar(rel_inf(M.precond_apply(pr, v, transpose=True, qr=True, dt=dt), ref_p)))
        print("QR adjoint", kind, prec, "errors", e, "bars", bars)
        assert e[0] <= bars[0] and e[1] <= bars[1]
        plan.close()
