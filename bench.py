"""Benchmark: one-body-preconditioned MFS mobility solve on one MI355X.

A step is one whole solve of the hot path on a resident plan: completion
strengths and right-hand side (pair sum over all pairs), GMRES on the square
preconditioned system (each matvec = pseudo-inverse blocks on the matrix
cores, FP64 rigid-body projection, off-body pair sum, + gamma), the FP64
true-residual check, and recovery of the rigid velocities.  Inputs are
resident in HBM before the timed region starts; the per-shape factorisation
is setup and is timed separately.

Printed JSON line (one):
  value       - pair interactions evaluated per second over the timed steps
                (off-body pairs x matvecs + all pairs of the right-hand side),
                whole-job, mixed precision, in Ginteractions/s
  roofline    - the dominant kernel (mixed Stokes pair sum): 28 flops per pair
                x pairs per launch / average launch time from HIP events on
                its own stream during the timed steps, against the FP32
                vector peak
  cpu_baseline- the FP64 CPU oracle on a bounded sample of the same workload
  extra       - FP64 solve time on the GPU, speedup, iteration counts, ...

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = {1: 28.0, 0: 11.0}      # Stokes, Laplace (FMA = 2, rsqrt = 1)
PEAK_FP32_TFLOPS = 157.3                  # MI355X FP32 vector peak (published)
STOP_FACTOR = 0.1                         # the library's default GMRES stopping margin
WORKLOADS = ("ellipsoids_100", "ellipsoids_1000", "batched_64", "spheres_200_grad", "ellipsoids_100_2way",
             "ellipsoids_10000")
# minutes-long solves: one step, no warm-up, no autotuning, no separate FP64 solve, progress lines
LARGE = ("ellipsoids_10000",)


def _trace_marker(torch):
    """A kernel of its own name (torch's spin_kernel, a few hundred cycles, outside the timed region's
    clock) that brackets the timed steps in a kernel trace, so a profile can pick out exactly the
    launches the HIP events timed."""
    torch.cuda._sleep(100)


def _workload(name: str, kind: int):
    import mfs_workloads as W
    if name == "ellipsoids_100":
        return W.ellipsoids_100(kind)
    if name == "ellipsoids_1000":
        return W.ellipsoids_1000(kind)
    if name == "batched_64":
        return W.batched_64()
    if name == "spheres_200_grad":
        return W.spheres_200()
    if name == "ellipsoids_100_2way":
        return W.ellipsoids_100(1)
    if name == "ellipsoids_10000":
        return W.ellipsoids_10000(kind)
    raise SystemExit(f"unknown workload {name}; choose from {WORKLOADS}")


def _pairs_per_system(wl):
    """Per system: (kind, off-body pairs of one matvec, all pairs of the right-hand side)."""
    out = []
    for s in range(wl.n_sys):
        b0, b1 = int(wl.sys_body_ptr[s]), int(wl.sys_body_ptr[s + 1])
        n_src = [wl.shapes[wl.shape_of_body[b]].src.shape[0] for b in range(b0, b1)]
        n_trg = [wl.shapes[wl.shape_of_body[b]].trg.shape[0] for b in range(b0, b1)]
        tot = sum(n_src)
        out.append((int(wl.sys_kind[s]), float(sum(t * (tot - q) for t, q in zip(n_trg, n_src))),
                    float(sum(n_trg) * tot)))
    return out


def _counter_file(workload: str, kind: int) -> str:
    if workload == "batched_64":
        return os.path.join(ROOT, "profiles", "p2p_mixed_batched_64_pmc.txt")
    return os.path.join(ROOT, "profiles", f"p2p_mixed_{'stokes' if kind else 'laplace'}_{workload}_pmc.txt")


def _counter_traffic(workload: str, kind: int, shape):
    """HBM bytes per launch of the pair kernel at launch shape `shape` (targets
    per lane, work items, persistent) from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-kernel calibrated), or None when there is none for
    this workload or the kernel source has changed since the counters were taken."""
    import hashlib
    path = _counter_file(workload, kind)
    src = os.path.join(ROOT, "paper_2409_04215_amd", "csrc", "p2p_kernels.hip")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("machine-readable: "):
            rec = json.loads(line[len("machine-readable: "):])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if not rec or rec.get("source_sha256_16") != sha:
        return None
    for r in rec.get("per_shape", []):
        if tuple(r["launch"]) == tuple(shape):
            return r
    return None


GOLDEN = os.path.join(ROOT, "tests", "golden")
STORED = {("ellipsoids_100", 1): "ellipsoids_100_stokes_U.txt", ("ellipsoids_100", 0): "ellipsoids_100_laplace_phi.txt",
          ("ellipsoids_1000", 1): "ellipsoids_1000_stokes_U.txt", ("ellipsoids_1000", 0): "ellipsoids_1000_laplace_phi.txt"}


def _stored_oracle(workload: str, kind: int, wl):
    """Stored FP64 oracle outputs of this workload (GMRES tol 1e-10, written by
    tests/golden/make_golden.py): a list of (system, reference (P_s, 6) or (P_s,)),
    empty when none are stored."""
    import numpy as np
    if workload == "batched_64":
        path = os.path.join(GOLDEN, "batched_64_subset.txt")
        if not os.path.exists(path):
            return []
        tab = np.loadtxt(path, ndmin=2)
        out = []
        for sy in sorted(set(tab[:, 0].astype(int))):
            rows = tab[tab[:, 0] == sy]
            out.append((sy, rows[:, 2:8] if wl.sys_kind[sy] == 1 else rows[:, 2]))
        return out
    name = STORED.get((workload, kind))
    if name is None or not os.path.exists(os.path.join(GOLDEN, name)):
        return []
    return [(0, np.loadtxt(os.path.join(GOLDEN, name)).reshape(wl.n_body, -1).squeeze())]


def _vs_oracle(out, wl, stored):
    """Largest per-system rel_inf = max|out - ref| / max|ref| over the stored
    systems, separately for rigid velocities and potentials."""
    import numpy as np
    if not stored:
        return None
    dims = [6 if k == 1 else 1 for k in wl.sys_kind]
    offs = np.concatenate([[0], np.cumsum([dims[sy] * (wl.sys_body_ptr[sy + 1] - wl.sys_body_ptr[sy])
                                           for sy in range(wl.n_sys)])]).astype(np.int64)
    o = out.detach().cpu().numpy()
    res = {"systems": len(stored), "bodies": int(sum(len(r) for _, r in stored))}
    for sy, ref in stored:
        got = o[offs[sy]:offs[sy + 1]].reshape(ref.shape)
        key = "stokes_U" if wl.sys_kind[sy] == 1 else "laplace_phi"
        res[key] = max(res.get(key, 0.0), float(np.abs(got - ref).max() / np.abs(ref).max()))
    return res


def _kind_subset(wl, kind):
    """Points and structure of the systems of one kind (for the standalone pair sums)."""
    import numpy as np
    X, _ = wl.world_points("trg")
    Y, _ = wl.world_points("src")
    n_trg = np.array([wl.shapes[i].trg.shape[0] for i in wl.shape_of_body])
    n_src = np.array([wl.shapes[i].src.shape[0] for i in wl.shape_of_body])
    t_off = np.concatenate([[0], np.cumsum(n_trg)])
    s_off = np.concatenate([[0], np.cumsum(n_src)])
    sys_ptr, bodies = [0], []
    for sy in range(wl.n_sys):
        if wl.sys_kind[sy] == kind:
            b0, b1 = int(wl.sys_body_ptr[sy]), int(wl.sys_body_ptr[sy + 1])
            bodies += list(range(b0, b1))
            sys_ptr.append(len(bodies))
    if not bodies:
        return None
    bodies = np.array(bodies)
    xi = np.concatenate([np.arange(t_off[b], t_off[b + 1]) for b in bodies])
    yi = np.concatenate([np.arange(s_off[b], s_off[b + 1]) for b in bodies])
    return (np.array(sys_ptr, np.int64), np.concatenate([[0], np.cumsum(n_trg[bodies])]).astype(np.int64),
            np.concatenate([[0], np.cumsum(n_src[bodies])]).astype(np.int64), X[xi], Y[yi])


def standalone_p2p(mfs, torch, np, wl, per_sys, reps: int = 10, warm: int = 5):
    """The standalone pair sums (mfs_p2p_stokes, mfs_p2p_laplace; mixed, off-body
    pairs) on the workload's own points, one call per PDE kind over all its
    systems: HIP events on the calling stream around `reps` calls after `warm`
    untimed calls (the first builds the cached work tables; the others let the
    clocks settle after the host-side setup: at ellipsoids_100 the first five
    calls after it took 1.35 down to 1.24 ms, later ones 1.17 ms)."""
    res = {}
    for kind, fn in ((1, mfs.p2p_stokes), (0, mfs.p2p_laplace)):
        sub = _kind_subset(wl, kind)
        if sub is None:
            continue
        sp, tp, pp, X, Y = sub
        dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
        x, y = dev(X), dev(Y)
        st = dev(np.random.default_rng(5).standard_normal((Y.shape[0], 3) if kind else Y.shape[0]))
        out = torch.empty((X.shape[0], 3) if kind else X.shape[0], dtype=torch.float64, device="cuda")
        for _ in range(warm):
            fn(sp, tp, pp, x, y, st, out=out)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn(sp, tp, pp, x, y, st, out=out)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        pairs = sum(off for k, off, _ in per_sys if k == kind)
        res["stokes" if kind else "laplace"] = {"ms_per_call": round(ms, 4), "ginter_s": round(pairs / (ms * 1e-3) / 1e9, 2),
                                                "off_body_pairs": pairs}
    return res


def _timed_solves(plan, net, tol, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its, res = [], []
    for _ in range(steps):
        out, info = plan.solve(net, tol=tol)
        its.append(int(info["iters"][0]))
        res.append(float(info["relres"][0]))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, its, res, out


def cpu_baseline(wl, budget_s: float = 15.0):
    """The oracle's FP64 matvec on a bounded sample of the workload: for one
    suspension the whole budget goes to it; for several (batched_64), half the
    budget each to the largest Stokes and the largest Laplace system, and the
    rate is their pairs over their summed time."""
    if wl.n_sys == 1:
        return _cpu_baseline_one(wl, budget_s)
    sizes = [int(wl.sys_body_ptr[sy + 1] - wl.sys_body_ptr[sy]) for sy in range(wl.n_sys)]
    picks = []
    for kind in (1, 0):
        idx = [sy for sy in range(wl.n_sys) if wl.sys_kind[sy] == kind]
        if idx:
            picks.append(max(idx, key=lambda sy: sizes[sy]))
    parts = [_cpu_baseline_one(wl.system(sy), budget_s / len(picks)) for sy in picks]
    pairs = sum(p["pairs"] for p in parts)
    dt = sum(p["seconds"] for p in parts)
    out = dict(parts[0])
    out.update(value=pairs / dt / 1e9, seconds=dt, pairs=pairs,
               sample="; ".join(f"system {sy} ({sizes[sy]} bodies, {'Stokes' if wl.sys_kind[sy] else 'Laplace'}): "
                                f"{p['sample']}" for sy, p in zip(picks, parts)))
    return out


def _cpu_baseline_one(wl, budget_s: float = 15.0):
    """The oracle's matvec (FP64, plain C pair loops on all host threads plus
    numpy pseudo-inverse blocks), timed for about budget_s seconds: whole
    matvecs when one fits in the budget, else one matvec restricted to a
    sample of target rows.  Reports off-body pairs per second."""
    import numpy as np

    import mfs_workloads as W
    from oracle import mfs_oracle as O

    pr = O.Problem.from_workload(wl)
    g = W.random_vector(pr.n_gamma, 1)
    n_rows_all = pr.X.shape[0]
    n_src = pr.Y.shape[0]
    src_per_body = pr.bodies[0].Y.shape[0]
    rng = np.random.default_rng(0)

    def timed(rows):
        t0 = time.perf_counter()
        pr.matvec(g, rows=rows)
        return time.perf_counter() - t0

    # cost model t(rows) = fixed (pseudo-inverse blocks) + per_row * rows, from two sample sizes
    timed(np.arange(min(64, n_rows_all)))  # warm-up (thread pool, library load)
    r1, r2 = min(200, n_rows_all), min(2000, n_rows_all)
    t1 = timed(np.sort(rng.choice(n_rows_all, r1, replace=False)))
    t2 = timed(np.sort(rng.choice(n_rows_all, r2, replace=False)))
    per_row = max((t2 - t1) / max(r2 - r1, 1), 1e-9)
    fixed = max(t1 - per_row * r1, 0.0)
    full = fixed + per_row * n_rows_all
    if full <= budget_s:
        reps = 0
        t0 = time.perf_counter()
        while reps == 0 or time.perf_counter() - t0 < budget_s:
            pr.matvec(g)
            reps += 1
        dt = time.perf_counter() - t0
        pairs = reps * n_rows_all * (n_src - src_per_body)
        sample = (f"{reps} whole FP64 oracle matvec{'s' if reps > 1 else ''} of {wl.name} ({n_rows_all} collocation rows x "
                  f"{n_src - src_per_body} off-body sources each, plus all {len(pr.bodies)} pseudo-inverse "
                  f"blocks), {dt:.1f} s")
    else:
        n_rows = int(min(n_rows_all, max(r2, (budget_s - fixed) / per_row)))
        rows = np.sort(rng.choice(n_rows_all, n_rows, replace=False))
        dt = timed(rows)
        pairs = n_rows * (n_src - src_per_body)
        sample = (f"one FP64 oracle matvec of {wl.name} restricted to {n_rows} of {n_rows_all} collocation "
                  f"rows (all {len(pr.bodies)} pseudo-inverse blocks + those rows' off-body pair sums), "
                  f"{dt:.1f} s")
    return dict(value=pairs / dt / 1e9, unit="Ginteractions/s", cores=O.oracle_threads(), kind="oracle",
                sample=sample + "; off-body pairs per second of that work", seconds=dt, pairs=pairs,
                host_cpu=_cpu_model(), host_logical_cpus=os.cpu_count())


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def two_way_bench(args, mfs, torch, np):
    """The 2-way test (eq. (2way)) on ellipsoids_100 (Stokes): a step is one
    resistance solve (seeded rigid velocities U_ref -> forces F, proxies at the
    resistance scale) followed by one mobility solve (F -> U, proxies at 0.7).
    Reports eps_2way = |U - U_ref|_inf / |U_ref|_inf in both precisions."""
    import mfs_workloads as W
    wl = W.ellipsoids_100(W.STOKES)
    wr = W.with_proxy_scale(wl, W.resistance_proxy_scale())
    U_ref = np.random.default_rng(np.random.SeedSequence(7100)).standard_normal((wl.n_body, 6))
    u_ref = torch.tensor(U_ref.reshape(-1), dtype=torch.float64, device="cuda")
    off = float(sum(wl.shapes[0].trg.shape[0] for _ in range(wl.n_body)) * (wl.n_body - 1) * wl.shapes[0].src.shape[0])
    plans = {}
    for prec in (mfs.MIXED, mfs.FP64):
        res = mfs.Plan.from_workload(wr, prec, formulation=mfs.RESISTANCE)
        mob = mfs.Plan.from_workload(wl, prec)
        if not args.no_autotune:
            res.autotune(prec, reps=2)
            mob.autotune(prec, reps=2)
        plans[prec] = (res, mob)

    def step(prec):
        res, mob = plans[prec]
        F, ir = res.solve(u_ref, tol=args.tol)
        rmx, r64 = res.last_solve()
        U, im = mob.solve(F, tol=args.tol)
        mmx, m64 = mob.last_solve()
        mv = int(rmx[0] + r64[0] + mmx[0] + m64[0])
        pairs = mv * off + wl.n_body * wl.shapes[0].trg.shape[0] * wl.n_body * wl.shapes[0].src.shape[0]
        eps = float((U - u_ref).abs().max() / u_ref.abs().max())
        return eps, pairs, (int(ir["iters"][0]), int(im["iters"][0])), (int(rmx[0]), int(mmx[0]))

    out = {}
    for prec, steps in ((mfs.MIXED, args.steps), (mfs.FP64, args.fp64_steps)):
        for _ in range(args.warmup):
            step(prec)
        res, mob = plans[prec]
        if prec == mfs.MIXED:
            for p in (res, mob):
                p.set_timing(True)
                p.timing(mfs.MIXED, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tot = 0.0
        for _ in range(steps):
            eps, pairs, its, mx = step(prec)
            tot += pairs
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[prec] = dict(step_s=dt, eps=eps, pairs=tot / steps, iters=its, mixed_mv=mx)
        if prec == mfs.MIXED:
            n1, ms1, _ = res.timing(mfs.MIXED)
            n2, ms2, _ = mob.timing(mfs.MIXED)
            for p in (res, mob):
                p.set_timing(False)
            out["avg_ms"] = (ms1 + ms2) / max(n1 + n2, 1)
            out["launches"] = n1 + n2
    mx, f64 = out[mfs.MIXED], out[mfs.FP64]
    achieved = FLOPS_PER_PAIR[1] * off / (out["avg_ms"] * 1e-3) / 1e12
    rec = {
        "metric": "P2P Ginteractions/s + GMRES-to-1e-5 solve time, mixed vs FP64, 1 GPU",
        "value": round(mx["pairs"] / mx["step_s"] / 1e9, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(mx["step_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 pairs + f64",
        "data": "synthetic (seeded prolate spheroids; no dataset)",
        "config": {"workload": "ellipsoids_100_2way", "bodies": wl.n_body, "proxies_per_body": 400,
                   "collocation_per_body": 800, "kernel": "stokes resistance then mobility",
                   "gmres_tol": args.tol, "resistance_proxy_scale": round(W.resistance_proxy_scale(), 6),
                   "mobility_proxy_scale": 0.7},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
                     "kernel": "p2p_mixed_kernel (matvec pair sum)", "avg_launch_ms": round(out["avg_ms"], 4),
                     "launches": out["launches"]},
        "eps_2way_mixed": mx["eps"], "eps_2way_fp64": f64["eps"],
        "iters_resistance_mobility_mixed": mx["iters"], "iters_resistance_mobility_fp64": f64["iters"],
        "step_time_fp64_s": round(f64["step_s"], 5), "speedup_mixed_vs_fp64": round(f64["step_s"] / mx["step_s"], 3),
    }
    print(json.dumps(rec))
    return 0


# (targets per lane, work items, persistent grid): the autotuner's candidates
LAUNCH_SHAPES = [(tpl, items, per) for per in (0, 1) for tpl in (1, 2) for items in (1024, 2048, 4096, 8192, 16384)]


def counter_sweep(plan, mfs, torch, np):
    n = (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.mul(a, 1.0, out=b)  # one elementwise kernel that reads and writes 1 GiB
    torch.cuda.synchronize()
    del a, b
    g = torch.tensor(np.random.default_rng(3).standard_normal(plan.n_gamma), dtype=torch.float64, device="cuda")
    for tpl, items, per in LAUNCH_SHAPES:
        plan.set_launch(tpl, items, bool(per))
        plan.matvec(g, mfs.MIXED)
        torch.cuda.synchronize()
    plan.set_launch(1, 16384, False)
    plan.matvec(g, mfs.FP64)  # one FP64 matvec for the FP64 pair-kernel counters
    torch.cuda.synchronize()
    print(json.dumps({"counter_sweep": LAUNCH_SHAPES, "fp64_matvec_shape": [1, 16384, 0],
                      "calib_copy_bytes": 1 << 30}))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 5; 1 for the 10^4 case)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 1; 0 for the 10^4 case)")
    ap.add_argument("--workload", default="batched_64", choices=WORKLOADS,
                    help="default: batched_64, the largest single-GPU configuration (64 suspensions, 6917 bodies)")
    ap.add_argument("--kind", default="stokes", choices=("stokes", "laplace"),
                    help="PDE of the ellipsoid workloads (batched_64 mixes both; spheres_200_grad is Stokes)")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--fp64-steps", type=int, default=None,
                    help="FP64 solves timed for the speedup (default 2; 0 for the 10^4 case)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default pair-sum launch shape")
    ap.add_argument("--counter-sweep", action="store_true",
                    help="for rocprofv3 counter runs: one 1 GiB copy (calibration), one mixed matvec per "
                         "pair-sum launch shape the autotuner can pick (LAUNCH_SHAPES order), then one FP64 "
                         "matvec; prints the shapes")
    ap.add_argument("--launch", default=None,
                    help="fix the pair-sum launch shape instead of autotuning: TPL,WORK_ITEMS,PERSISTENT "
                         "(e.g. 1,16384,0; used for counter runs, which must repeat one shape)")
    ap.add_argument("--factorization", default="svd", choices=("svd", "qr"),
                    help="one-body factorisation of the plans: rocSOLVER SVD or the library's Householder QR")
    args = ap.parse_args()
    large = args.workload in LARGE
    args.steps = args.steps if args.steps is not None else (1 if large else 5)
    args.warmup = args.warmup if args.warmup is not None else (0 if large else 1)
    args.fp64_steps = args.fp64_steps if args.fp64_steps is not None else (0 if large else 2)
    if large:
        args.no_cpu = True
        args.no_autotune = True
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not built)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2409_04215_amd import mfs

    torch.cuda.set_device(0)
    if args.workload == "ellipsoids_100_2way":
        return two_way_bench(args, mfs, torch, np)
    kind = 0 if args.kind == "laplace" else 1
    grad = args.workload == "spheres_200_grad"
    wl = _workload(args.workload, kind)
    per_sys = _pairs_per_system(wl)
    net = torch.tensor(np.concatenate([n.reshape(-1) for n in wl.net]), dtype=torch.float64, device="cuda")

    t0 = time.perf_counter()
    fact = mfs.FACTOR_QR if args.factorization == "qr" else mfs.FACTOR_SVD
    plan_mx = mfs.Plan.from_workload(wl, mfs.MIXED, factorization=fact)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if args.counter_sweep:
        return counter_sweep(plan_mx, mfs, torch, np)
    plan_64 = mfs.Plan.from_workload(wl, mfs.FP64, factorization=fact) if args.fp64_steps > 0 else None
    max_iter = 100 if large else 200
    if large:
        t_start = time.perf_counter()

        def report(mv, active, relres):
            print(f"[solve] matvec {mv}: max relative residual estimate {relres:.3e}, "
                  f"{time.perf_counter() - t_start:.0f} s", file=sys.stderr, flush=True)

        plan_mx.set_progress(report)

    tuned = None
    if args.launch:
        tpl, items, per = (int(v) for v in args.launch.split(","))
        for p in (plan_mx, plan_64):
            if p is not None:
                p.set_launch(tpl, items, bool(per))
        tuned = (-tpl if per else tpl, items, float("nan"))
    elif not args.no_autotune:
        tuned = plan_mx.autotune(mfs.MIXED, reps=3)
        if plan_64 is not None:
            plan_64.autotune(mfs.FP64, reps=2)

    def step(plan):
        out, info = plan.solve(net, tol=args.tol, max_iter=max_iter)
        mx, f64 = plan.last_solve()
        pairs = sum((m + f) * off + rhs for (k, off, rhs), m, f in zip(per_sys, mx, f64))
        flops_mx = sum(m * off * FLOPS_PER_PAIR[k] for (k, off, rhs), m in zip(per_sys, mx))
        pairs_mx = sum(m * off for (k, off, rhs), m in zip(per_sys, mx))
        its = info["iters"]
        if grad:
            g, _, _, _, _ = plan.gmres_solve_backward(info["gamma"], info["s0"], 2.0 * out, tol=args.tol)
            amx, af64 = plan.last_solve()
            # adjoint matvecs (transposed pair sums) + the two position-gradient passes
            pairs += sum((m + f + 2) * off for (k, off, rhs), m, f in zip(per_sys, amx, af64))
            its = np.concatenate([its, amx + af64])
        return out, info, pairs, flops_mx, pairs_mx, its

    for _ in range(args.warmup):
        step(plan_mx)
    plan_mx.set_timing(True)
    plan_mx.timing(mfs.MIXED, reset=True)
    plan_mx.timing(mfs.FP64, reset=True)
    _trace_marker(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_pairs = tot_flops = tot_pairs_mx = 0.0
    for _ in range(args.steps):
        out_mx, info_mx, pairs, flops, pairs_mx, its = step(plan_mx)
        tot_pairs += pairs
        tot_flops += flops
        tot_pairs_mx += pairs_mx
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / args.steps
    _trace_marker(torch)
    n_mx, ms_mx, ppl = plan_mx.timing(mfs.MIXED)
    n_chk, ms_chk, _ = plan_mx.timing(mfs.FP64)
    plan_mx.set_timing(False)
    value = tot_pairs / args.steps / step_s / 1e9

    # the same solves replayed from the captured matvec graph (after the timed region: the kernel
    # events of the timed region keep graphs off)
    graph_s = None
    if not large:
        plan_mx.set_graph(True)
        step(plan_mx)
        torch.cuda.synchronize()
        n_graph = min(args.steps, 3)
        t0 = time.perf_counter()
        for _ in range(n_graph):
            step(plan_mx)
        torch.cuda.synchronize()
        graph_s = (time.perf_counter() - t0) / n_graph
        plan_mx.set_graph(False)

    fp64_s = diff = None
    info_64 = None
    n64, ms64 = n_chk, ms_chk  # FP64 pair rate from the true-residual checks unless FP64 solves run
    if plan_64 is not None:
        plan_64.solve(net, tol=args.tol, max_iter=max_iter)
        plan_64.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.fp64_steps):
            out_64, info_64, _, _, _, _ = step(plan_64)
        torch.cuda.synchronize()
        fp64_s = (time.perf_counter() - t0) / args.fp64_steps
        n64, ms64, _ = plan_64.timing(mfs.FP64)
        plan_64.set_timing(False)
        diff = float((out_mx - out_64).abs().max() / out_64.abs().max())
    extra = {}
    stored = _stored_oracle(args.workload, kind, wl)
    if stored:
        extra["rel_inf_vs_oracle_mixed"] = _vs_oracle(out_mx, wl, stored)
        if info_64 is not None:
            extra["rel_inf_vs_oracle_fp64"] = _vs_oracle(out_64, wl, stored)
    if not large:
        # the same mixed solve under the stopping rule as the paper states it (stop once the
        # residual estimate is below tol): fewer iterations, larger output error
        plan_mx.set_stop_factor(1.0)
        step(plan_mx)
        torch.cuda.synchronize()
        n_s1 = min(args.steps, 3)
        t0 = time.perf_counter()
        for _ in range(n_s1):
            out_s1, info_s1, _, _, _, its_s1 = step(plan_mx)
        torch.cuda.synchronize()
        extra["stop_factor_1"] = {"solve_time_mixed_s": round((time.perf_counter() - t0) / n_s1, 5),
                                  "max_iters": int(np.max(its_s1)),
                                  "rel_inf_vs_oracle": _vs_oracle(out_s1, wl, stored) if stored else None}
        plan_mx.set_stop_factor(STOP_FACTOR)
    if not large:
        extra["p2p_standalone_mixed"] = standalone_p2p(mfs, torch, np, wl, per_sys)
    # moving the bodies of the resident plan (same positions here) against building a new one:
    # the one-body factors are kept, only the geometry is rebuilt
    t_mv = time.perf_counter()
    plan_mx.set_bodies(wl.centre, wl.rot)
    extra["move_bodies_s"] = round(time.perf_counter() - t_mv, 4)
    if wl.n_sys == 1:
        # the paper's accuracy diagnostic (eq. (residual)) at 1732 points per body surface, after the timed region
        import mfs_workloads as W
        _, sig = plan_mx.extract(info_mx["gamma"], info_mx["s0"], want_sigma=True)
        t_res = time.perf_counter()
        eps = plan_mx.surface_residual(sig, out_mx, [W.surface_test_points(sh) for sh in wl.shapes]).cpu().numpy()
        # Stokes: pointwise |u - g| / |g|, which grows without bound where the rigid velocity g nearly
        # vanishes, so the 99th percentile and the median are reported beside the maximum.
        # Laplace: the absolute error |u - phi| against the body potential.
        extra["surface_residual"] = {"measure": "relative" if kind == 1 else "absolute",
                                     "max": float(eps.max()), "p99": float(np.percentile(eps, 99)),
                                     "median": float(np.median(eps)), "points_per_body": 1732}
        extra["surface_residual_s"] = round(time.perf_counter() - t_res, 3)
    if large and kind == 1:
        # exact net force and torque of the strengths (eq. (force_syst)): a property of the solve
        _, sigma = plan_mx.extract(info_mx["gamma"], info_mx["s0"], want_sigma=True)
        Y, sb = wl.world_points("src")
        sg = sigma.cpu().numpy().reshape(-1, 3)
        F = np.zeros((wl.n_body, 3))
        T = np.zeros((wl.n_body, 3))
        np.add.at(F, sb, sg)
        np.add.at(T, sb, np.cross(Y - wl.centre[sb], sg))
        want = wl.net[0]
        extra["net_force_torque_mismatch"] = float(np.abs(np.concatenate([F, T], 1) - want).max() / np.abs(want).max())
        extra["context"] = ("the paper solves 10^4 Type T ellipsoids (delta 0.2, N_v 34) on one CPU workstation "
                            "with an FMM in under two hours")

    shape = (abs(tuned[0]), tuned[1], int(tuned[0] < 0)) if tuned else (1, 2048, 0)
    traffic = _counter_traffic(args.workload, kind, shape)
    avg_ms = ms_mx / max(n_mx, 1)
    achieved = tot_flops / (ms_mx * 1e-3) / 1e12 if ms_mx > 0 else 0.0
    flops_per_pair = tot_flops / max(tot_pairs_mx, 1.0)
    kinds = sorted(set(k for k, _, _ in per_sys))
    kind_name = {0: "laplace elastance", 1: "stokes mobility"}
    off_total = sum(off for _, off, _ in per_sys)
    rec = {
        "metric": "P2P Ginteractions/s + GMRES-to-1e-5 solve time, mixed vs FP64, 1 GPU",
        "value": round(value, 3),
        "unit": "Ginteractions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 pairs / f64 accumulation, projection and GMRES",
        "data": "synthetic (seeded random suspensions; the paper publishes no cluster files)",
        "config": {"workload": args.workload, "systems": wl.n_sys, "bodies": wl.n_body,
                   "proxies_per_body": int(wl.shapes[0].src.shape[0]),
                   "collocation_per_body": int(wl.shapes[0].trg.shape[0]),
                   "kernel": " + ".join(kind_name[k] for k in kinds) + (" + centre gradient" if grad else ""),
                   "gmres_tol": args.tol,
                   "gmres_stop": (f"estimate <= {STOP_FACTOR}*tol (mfs_plan_set_stop_factor), then FP64 true residual "
                                  f"<= {STOP_FACTOR}*tol by refinement (converged when <= tol)"),
                   "unknowns_gamma": plan_mx.n_gamma, "off_body_pairs_per_matvec": off_total,
                   "factorization": args.factorization},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": round(traffic["traffic_bytes"]) if traffic else None,
                     "traffic_fetch_bytes": round(traffic["fetch_bytes"]) if traffic else None,
                     "traffic_write_bytes": round(traffic["write_bytes"]) if traffic else None,
                     "kernel": "p2p_mixed_kernel (matvec pair sum)", "avg_launch_ms": round(avg_ms, 4),
                     "launches": n_mx, "flops_per_pair": round(flops_per_pair, 3),
                     "flops_per_launch": tot_flops / max(n_mx, 1)},
        "solve_time_mixed_s": round(step_s, 5),
        "solve_time_mixed_graph_s": round(graph_s, 5) if graph_s else None,
        "solve_time_fp64_s": round(fp64_s, 5) if fp64_s else None,
        "speedup_mixed_vs_fp64": round(fp64_s / step_s, 3) if fp64_s else None,
        "matvecs_per_step_mixed": (n_mx + n_chk) / args.steps,
        "fp64_check_matvecs_per_step": n_chk / args.steps,
        "iters_per_system_last_step": [int(x) for x in np.asarray(its).reshape(-1)][:128],
        "relres_mixed_true_fp64_max": float(np.max(info_mx["relres"])),
        "relres_fp64_max": float(np.max(info_64["relres"])) if info_64 else None,
        "p2p_kernel_ginter_s_mixed": round(tot_pairs_mx / (ms_mx * 1e-3) / 1e9, 2) if ms_mx > 0 else None,
        "p2p_kernel_ginter_s_fp64": round(ppl * n64 / (ms64 * 1e-3) / 1e9, 2) if ms64 > 0 and wl.n_sys == 1 else None,
        "rel_diff_out_mixed_vs_fp64_gpu": diff,
        "setup_s": round(setup_s, 3),
        "autotuned_launch": {"targets_per_lane": abs(tuned[0]), "work_items": tuned[1],
                             "persistent_grid": tuned[0] < 0} if tuned else None,
        **extra,
    }
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
