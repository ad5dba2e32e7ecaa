"""Writes stored oracle results (FP64, GMRES tol 1e-10) to text files next to
this script.  Calls only oracle/ and the seeded input generators.

    python tests/golden/make_golden.py            # ellipsoids_100 mobility / elastance (minutes)
    python tests/golden/make_golden.py two_way    # ellipsoids_100 resistance -> mobility (2-way error)
    python tests/golden/make_golden.py e100_tight # ellipsoids_100 at GMRES tol 1e-13 (minutes)
    python tests/golden/make_golden.py rows_10000 # 10^4 Type T case: 1000 sampled rows (tens of minutes)
    python tests/golden/make_golden.py rows_10000_model  # the float32 model on 100 of those rows
    python tests/golden/make_golden.py rows_10000_model64 rows_1000_model64  # the float64 model of the stored rows
    python tests/golden/make_golden.py rows_1000  # ellipsoids_1000: 2000 sampled rows, oracle and float32 model
    python tests/golden/make_golden.py batched    # batched_64: a stated subset of the 64 systems (~1.5 h)
    python tests/golden/make_golden.py e1000_laplace | e1000_stokes   # ellipsoids_1000 (~1 h / ~4 h)
    python tests/golden/make_golden.py grad_200   # spheres_200: the adjoint gradients (~1 h)

The long runs set MFS_ORACLE_NATIVE=1 (the oracle's C loops built with
-O3 -march=native; same source) to fit in hours on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mfs_workloads as W  # noqa: E402
from oracle import fp32_model as M  # noqa: E402
from oracle import mfs_oracle as O  # noqa: E402

TOL = 1e-10
# batched_64: the systems stored are every system of at most this many bodies
# plus the largest system of each kind.
BATCHED_SMALL = 150


def _log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def _logged(pr, what):
    """The oracle's matvec with one log line per call (progress of hour-long solves)."""
    count = [0]
    t0 = time.time()

    def mv(g):
        count[0] += 1
        out = pr.matvec(g)
        _log(f"{what}: matvec {count[0]} done, {time.time() - t0:.0f} s")
        return out
    return mv


def _solve(pr, net, what):
    """Problem.solve with a progress line per matvec (same steps: rhs, GMRES, extract)."""
    t0 = time.time()
    b, s0 = pr.rhs(net)
    _log(f"{what}: right-hand side done, {time.time() - t0:.0f} s")
    gamma, iters, hist = O.gmres(_logged(pr, what), b, TOL)
    out, lam, sigma = pr.extract(gamma, s0)
    return dict(out=out, iters=iters, hist=hist, secs=time.time() - t0)


def two_way():
    """Resistance solve of ellipsoids_100 (proxies at the resistance scale) with
    seeded rigid velocities U_ref, then the mobility solve (proxies at 0.7)
    with the resulting forces: stores U_ref, F and U (eq. (2way))."""
    wl = W.ellipsoids_100(W.STOKES)
    wr = W.with_proxy_scale(wl, W.resistance_proxy_scale())
    U_ref = np.random.default_rng(np.random.SeedSequence(7100)).standard_normal((wl.n_body, 6))
    t0 = time.time()
    r = O.two_way_error(O.ResistanceProblem.from_workload(wr), O.Problem.from_workload(wl), U_ref, tol=TOL)
    dt = time.time() - t0
    hdr = (f"2-way test of the seeded ellipsoids_100 workload: columns U_ref (6), F (6), U (6) per body;\n"
           f"resistance proxies at scale {W.resistance_proxy_scale():.6f}, mobility at 0.7; U_ref from "
           f"SeedSequence(7100); FP64 oracle, GMRES tol 1e-10,\n"
           f"{r['iters_res']} resistance + {r['iters_mob']} mobility iterations, {dt:.0f} s; eps_2way = "
           f"{r['eps']:.6e}.  Written by tests/golden/make_golden.py two_way (oracle only).")
    np.savetxt(os.path.join(HERE, "ellipsoids_100_two_way.txt"),
               np.concatenate([U_ref, r["F"].reshape(-1, 6), r["U"].reshape(-1, 6)], axis=1), fmt="%.17e", header=hdr)
    print("two_way", r["iters_res"], r["iters_mob"], r["eps"], f"{dt:.0f}s", flush=True)


def e100():
    for kind, name, what in ((W.STOKES, "ellipsoids_100_stokes_U.txt", "rigid velocities [v; omega] per body"),
                             (W.LAPLACE, "ellipsoids_100_laplace_phi.txt", "potentials per body")):
        wl = W.ellipsoids_100(kind)
        t0 = time.time()
        sol = O.Problem.from_workload(wl).solve(wl.net[0], tol=TOL)
        dt = time.time() - t0
        out = np.asarray(sol["out"]).reshape(wl.n_body, -1)
        hdr = (f"oracle solution of the seeded ellipsoids_100 workload ({'Stokes mobility' if kind else 'Laplace elastance'}),\n"
               f"{what}; FP64 oracle, GMRES tol 1e-10, {sol['iters']} iterations, {dt:.0f} s.\n"
               f"Written by tests/golden/make_golden.py (oracle only).")
        np.savetxt(os.path.join(HERE, name), out, fmt="%.17e", header=hdr)
        print(name, sol["iters"], f"{dt:.0f}s", flush=True)


def e100_tight():
    """ellipsoids_100 solved to GMRES tol 1e-13: a reference whose own stopping
    error lies far below that of a solve at tol 1e-10.  The header keeps the
    tol-1e-10 solve's final residual estimate rho and its output error
    against this reference, err: err / rho is the oracle's ratio of output
    error to relative residual near convergence, which sizes the FP64 bar of
    a solve at tol 1e-10 from the residual it ends at."""
    for kind, name in ((W.STOKES, "ellipsoids_100_stokes_U_tight.txt"), (W.LAPLACE, "ellipsoids_100_laplace_phi_tight.txt")):
        wl = W.ellipsoids_100(kind)
        pr = O.Problem.from_workload(wl)
        t0 = time.time()
        s10 = pr.solve(wl.net[0], tol=TOL)
        s13 = pr.solve(wl.net[0], tol=1e-13)
        dt = time.time() - t0
        out = np.asarray(s13["out"]).reshape(wl.n_body, -1)
        err = float(np.abs(np.asarray(s10["out"]) - np.asarray(s13["out"])).max() / np.abs(np.asarray(s13["out"])).max())
        hdr = (f"oracle solution of the seeded ellipsoids_100 workload ({'Stokes mobility' if kind else 'Laplace elastance'})"
               f" at GMRES tol 1e-13 ({s13['iters']} iterations, final residual estimate {s13['hist'][-1]:.3e});\n"
               f"tol-1e-10 solve: rho {s10['hist'][-1]:.6e} err {err:.6e} ({s10['iters']} iterations); {dt:.0f} s.\n"
               f"Written by tests/golden/make_golden.py e100_tight (oracle only).")
        np.savetxt(os.path.join(HERE, name), out, fmt="%.17e", header=hdr)
        _log(name, s13["iters"], s10["hist"][-1], err, f"{dt:.0f}s")


def e1000(kind):
    """Oracle solution of ellipsoids_1000 (Section 3.3 recovery, eqs. (vkal), (getU))."""
    name = "ellipsoids_1000_stokes_U.txt" if kind == W.STOKES else "ellipsoids_1000_laplace_phi.txt"
    wl = W.ellipsoids_1000(kind)
    pr = O.Problem.from_workload(wl)
    sol = _solve(pr, wl.net[0], f"ellipsoids_1000 kind {kind}")
    out = np.asarray(sol["out"]).reshape(wl.n_body, -1)
    hdr = (f"oracle solution of the seeded ellipsoids_1000 workload "
           f"({'Stokes mobility, [v; omega]' if kind else 'Laplace elastance, phi'} per body);\n"
           f"FP64 oracle (C loops built -O3 -march=native), GMRES tol {TOL:g}, {sol['iters']} iterations, "
           f"{sol['secs']:.0f} s on {O.oracle_threads()} threads; final residual estimate {sol['hist'][-1]:.3e}.\n"
           f"Written by tests/golden/make_golden.py (oracle only).")
    np.savetxt(os.path.join(HERE, name), out, fmt="%.17e", header=hdr)
    _log(name, sol["iters"], f"{sol['secs']:.0f}s")


def batched_subset(wl):
    """The stored subset of batched_64: every system of at most BATCHED_SMALL
    bodies, and the largest system of each kind."""
    sizes = np.diff(wl.sys_body_ptr)
    pick = [s for s in range(wl.n_sys) if sizes[s] <= BATCHED_SMALL]
    for kind in (W.LAPLACE, W.STOKES):
        idx = [s for s in range(wl.n_sys) if wl.sys_kind[s] == kind]
        pick.append(max(idx, key=lambda s: sizes[s]))
    return sorted(set(pick), key=lambda s: (sizes[s], s))


def batched():
    """Oracle solutions of a subset of batched_64's suspensions, each solved on
    its own (the systems are independent).  Rows: system, body, then phi
    (Laplace, one column, padded with zeros) or [v; omega] (Stokes, six)."""
    wl = W.batched_64()
    sizes = np.diff(wl.sys_body_ptr)
    rows, notes = [], []
    path = os.path.join(HERE, "batched_64_subset.txt")
    t_all = time.time()
    for s in batched_subset(wl):
        pr = O.Problem.from_workload(wl, s)
        sol = _solve(pr, wl.net[s], f"batched_64 system {s} ({sizes[s]} bodies, kind {wl.sys_kind[s]})")
        out = np.asarray(sol["out"]).reshape(sizes[s], -1)
        pad = np.zeros((sizes[s], 6))
        pad[:, :out.shape[1]] = out
        rows.append(np.concatenate([np.full((sizes[s], 1), s), np.arange(sizes[s])[:, None], pad], axis=1))
        notes.append(f"{s}:{sol['iters']}")
        hdr = (f"oracle solutions of a subset of the seeded batched_64 workload: every system of at most "
               f"{BATCHED_SMALL} bodies and the largest of each kind.\n"
               f"Columns: system, body (within the system), then phi (Laplace; other columns 0) or [v; omega] (Stokes).\n"
               f"FP64 oracle (C loops built -O3 -march=native), each system solved alone, GMRES tol {TOL:g}; "
               f"system:iterations {' '.join(notes)}; {time.time() - t_all:.0f} s.\n"
               f"Written by tests/golden/make_golden.py batched (oracle only).")
        np.savetxt(path, np.concatenate(rows), fmt="%.17e", header=hdr)
        _log(f"system {s} stored, {sol['iters']} iterations")


def rows_10000():
    """The paper's 10^4 Type T case (Section 4.2): right-hand side and the matvec
    of a seeded random vector and of a seeded smooth field, on 1000 sampled
    collocation rows, each computed by the oracle over all sources."""
    t0 = time.time()
    wl = W.ellipsoids_10000(W.STOKES)
    pr = O.Problem.from_workload(wl)
    _log(f"10^4: workload and oracle set-up, {time.time() - t0:.0f} s")
    rows = np.sort(np.random.default_rng(86).choice(pr.X.shape[0], 1000, replace=False))
    g = W.random_vector(pr.n_gamma, 87)
    sm = W.smooth_vector(wl, 88)
    ref_b, _ = pr.rhs(wl.net[0], rows=rows)
    _log(f"10^4: right-hand side rows, {time.time() - t0:.0f} s")
    ref_g = pr.matvec(g, rows=rows)
    _log(f"10^4: matvec rows (random), {time.time() - t0:.0f} s")
    ref_sm = pr.matvec(sm, rows=rows)
    _log(f"10^4: matvec rows (smooth), {time.time() - t0:.0f} s")
    tab = np.concatenate([rows[:, None].astype(np.float64), ref_b.reshape(-1, 3), ref_g.reshape(-1, 3),
                          ref_sm.reshape(-1, 3)], axis=1)
    hdr = ("the seeded ellipsoids_10000 workload (10^4 Type T ellipsoids, N = 658, M = 842, Stokes):\n"
           "1000 collocation rows drawn by default_rng(86); columns: row, right-hand side b (3), "
           "A g (3) for g = random_vector(n_gamma, 87), A s (3) for s = smooth_vector(88).\n"
           f"FP64 oracle over all 6.58e6 proxies per row, {time.time() - t0:.0f} s.  "
           "Written by tests/golden/make_golden.py rows_10000 (oracle only).")
    np.savetxt(os.path.join(HERE, "ellipsoids_10000_rows.txt"), tab, fmt="%.17e", header=hdr)
    _log("10^4 rows stored")


def rows_1000():
    """ellipsoids_1000, both kinds: the right-hand side and the matvecs of a
    seeded random vector and of a seeded smooth field on 2000 sampled
    collocation rows, by the FP64 oracle and by its float32 model
    (oracle/fp32_model.py, which sizes the mixed bars)."""
    for kind, name in ((W.STOKES, "stokes"), (W.LAPLACE, "laplace")):
        t0 = time.time()
        wl = W.ellipsoids_1000(kind)
        pr = O.Problem.from_workload(wl)
        rows = np.sort(np.random.default_rng(81).choice(pr.X.shape[0], 2000, replace=False))
        g = W.random_vector(pr.n_gamma, 82)
        sm = W.smooth_vector(wl, 83)
        cols = [pr.rhs(wl.net[0], rows=rows)[0], pr.matvec(g, rows=rows), pr.matvec(sm, rows=rows)]
        _log(f"ellipsoids_1000 {name}: oracle rows, {time.time() - t0:.0f} s")
        cols += [M.rhs(pr, wl.net[0], rows=rows), M.matvec(pr, g, rows=rows), M.matvec(pr, sm, rows=rows)]
        _log(f"ellipsoids_1000 {name}: float32 model rows, {time.time() - t0:.0f} s")
        d = 3 if kind == W.STOKES else 1
        tab = np.concatenate([rows[:, None].astype(np.float64)] + [c.reshape(-1, d) for c in cols], axis=1)
        hdr = (f"the seeded ellipsoids_1000 workload ({name}): 2000 collocation rows drawn by default_rng(81);\n"
               f"columns: row, then ({d} each) the right-hand side b, A g for g = random_vector(n_gamma, 82), "
               f"A s for s = smooth_vector(83) by the FP64 oracle, then the same three by its float32 model.\n"
               f"{time.time() - t0:.0f} s.  Written by tests/golden/make_golden.py rows_1000 (oracle/ only).")
        np.savetxt(os.path.join(HERE, f"ellipsoids_1000_{name}_rows.txt"), tab, fmt="%.17e", header=hdr)


def rows_10000_model():
    """The float32 model of the 10^4 case's stored rows, on the first 100 of them."""
    t0 = time.time()
    tab = np.loadtxt(os.path.join(HERE, "ellipsoids_10000_rows.txt"))[:100]
    rows = tab[:, 0].astype(np.int64)
    wl = W.ellipsoids_10000(W.STOKES)
    pr = O.Problem.from_workload(wl)
    g = W.random_vector(pr.n_gamma, 87)
    sm = W.smooth_vector(wl, 88)
    cols = [M.rhs(pr, wl.net[0], rows=rows)]
    _log(f"10^4 model: right-hand side rows, {time.time() - t0:.0f} s")
    cols.append(M.matvec(pr, g, rows=rows))
    _log(f"10^4 model: matvec rows (random), {time.time() - t0:.0f} s")
    cols.append(M.matvec(pr, sm, rows=rows))
    out = np.concatenate([rows[:, None].astype(np.float64)] + [c.reshape(-1, 3) for c in cols], axis=1)
    hdr = ("the float32 model (oracle/fp32_model.py) of the first 100 stored rows of ellipsoids_10000_rows.txt;\n"
           "columns: row, right-hand side b (3), A g (3), A s (3) (the same vectors).\n"
           f"{time.time() - t0:.0f} s.  Written by tests/golden/make_golden.py rows_10000_model (oracle/ only).")
    np.savetxt(os.path.join(HERE, "ellipsoids_10000_model_rows.txt"), out, fmt="%.17e", header=hdr)
    _log("10^4 model rows stored")


GRAD_SAMPLE = (0, 37, 74, 111, 148, 185)  # spheres_200 bodies whose model gradients are stored


def _model_body_gradients(pr, info, bodies, dt):
    """dJ/dc and dJ/d[f; t] of the listed bodies by the model of precision dt
    (oracle/fp32_model.py): the pair sums that form them (all off-body pairs of
    the body's points; the transposed all-pairs sum for the net gradient),
    taken on the oracle's adjoint solution w and strengths sigma in `info`."""
    w = info["w"].reshape(-1, 3)
    sg = info["sol"]["sigma"].reshape(-1, 3)
    cen = np.stack([b.centre for b in pr.bodies])
    out_c, out_n = [], []
    for k in bodies:
        rt = pr.trg_body == k
        rs = pr.src_body == k
        gx, _ = M.pair_grad(pr.kind, pr.X[rt], pr.trg_body[rt], w[rt], pr.Y, pr.src_body, sg, cen, True, pr.mu, dt)
        _, gy = M.pair_grad(pr.kind, pr.X, pr.trg_body, w, pr.Y[rs], pr.src_body[rs], sg[rs], cen, True, pr.mu, dt)
        out_c.append(-(gx.sum(axis=0) + gy.sum(axis=0)))
        t = -M.pair_sum(pr.kind, pr.Y[rs], pr.src_body[rs], pr.X, pr.trg_body, w, cen, False, pr.mu, dt).reshape(-1)
        KN = O.K_matrix(pr.bodies[k].Y, pr.bodies[k].centre)
        out_n.append(np.linalg.solve(KN.T @ KN, KN.T @ t))
    return np.array(out_c), np.array(out_n)


def grad_200():
    """spheres_200 (200 unit spheres, N = 400, M = 800, Stokes mobility), J = sum |U|^2:
    the oracle's dJ/dc and dJ/d[f; t] with both of its solves at GMRES tol 1e-13 (the
    reference), 1e-12 and 1e-8, and the float32 and float64 models' gradients of the
    bodies GRAD_SAMPLE on the reference's adjoint solution and strengths."""
    t0 = time.time()
    wl = W.spheres_200()
    pr = O.Problem.from_workload(wl)
    res = {}
    for tol in (1e-13, 1e-12, 1e-8):
        J, g, info = pr.velocity_loss_gradient(wl.net[0], tol=tol)
        res[tol] = (J, g, info)
        _log(f"spheres_200 gradient at tol {tol:g}: J = {J:.16e}, {info['sol']['iters']} + {info['adj_iters']} "
             f"iterations, {time.time() - t0:.0f} s")
    cols = []
    for tol in (1e-13, 1e-12, 1e-8):
        cols += [res[tol][1], np.asarray(res[tol][2]["grad_net"]).reshape(-1, 6)]
    hdr = (f"the seeded spheres_200 workload (200 unit spheres, N = 400, M = 800, Stokes mobility), "
           f"J = sum |U|^2 = {res[1e-13][0]:.17e}:\n"
           f"per body dJ/dc (3) and dJ/d[f; t] (6) by the FP64 oracle with both solves at GMRES tol 1e-13, "
           f"then at 1e-12, then at 1e-8; {time.time() - t0:.0f} s.\n"
           f"Written by tests/golden/make_golden.py grad_200 (oracle only).")
    np.savetxt(os.path.join(HERE, "spheres_200_gradient.txt"), np.concatenate(cols, axis=1), fmt="%.17e", header=hdr)
    info = res[1e-13][2]
    mc32, mn32 = _model_body_gradients(pr, info, GRAD_SAMPLE, M.F32)
    _log(f"spheres_200 float32 model gradients, {time.time() - t0:.0f} s")
    mc64, mn64 = _model_body_gradients(pr, info, GRAD_SAMPLE, np.float64)
    _log(f"spheres_200 float64 model gradients, {time.time() - t0:.0f} s")
    tab = np.concatenate([np.array(GRAD_SAMPLE, np.float64)[:, None], mc32, mn32, mc64, mn64], axis=1)
    hdr = ("the float32 and float64 models (oracle/fp32_model.py) of the spheres_200 gradients of the bodies in the "
           "first column, on the oracle's tol-1e-13 adjoint solution and strengths:\n"
           "columns: body, dJ/dc (3) and dJ/d[f; t] (6) by the float32 model, then the same by the float64 model.\n"
           f"Written by tests/golden/make_golden.py grad_200 (oracle/ only).")
    np.savetxt(os.path.join(HERE, "spheres_200_gradient_model.txt"), tab, fmt="%.17e", header=hdr)
    _log("spheres_200 gradients stored")


def _model64_rows(pr, wl, rows, g, sm):
    """Right-hand side and both matvecs on `rows` by the float64 model
    (oracle/fp32_model.py with dt = float64: another summation order and an
    independent FP64 SVD of S_L), which sizes the FP64 bars."""
    F64 = np.float64
    return [M.rhs(pr, wl.net[0], rows=rows, dt=F64), M.matvec(pr, g, rows=rows, dt=F64),
            M.matvec(pr, sm, rows=rows, dt=F64)]


def rows_1000_model64():
    """The float64 model of ellipsoids_1000's stored rows (both kinds)."""
    for kind, name in ((W.STOKES, "stokes"), (W.LAPLACE, "laplace")):
        t0 = time.time()
        rows = np.loadtxt(os.path.join(HERE, f"ellipsoids_1000_{name}_rows.txt"))[:, 0].astype(np.int64)
        wl = W.ellipsoids_1000(kind)
        pr = O.Problem.from_workload(wl)
        cols = _model64_rows(pr, wl, rows, W.random_vector(pr.n_gamma, 82), W.smooth_vector(wl, 83))
        d = 3 if kind == W.STOKES else 1
        tab = np.concatenate([rows[:, None].astype(np.float64)] + [c.reshape(-1, d) for c in cols], axis=1)
        hdr = (f"the float64 model (oracle/fp32_model.py, dt = float64) of the rows of ellipsoids_1000_{name}_rows.txt;\n"
               f"columns: row, then ({d} each) b, A g, A s (the same vectors).\n"
               f"{time.time() - t0:.0f} s.  Written by tests/golden/make_golden.py rows_1000_model64 (oracle/ only).")
        np.savetxt(os.path.join(HERE, f"ellipsoids_1000_{name}_model64_rows.txt"), tab, fmt="%.17e", header=hdr)
        _log(f"ellipsoids_1000 {name} float64 model rows stored, {time.time() - t0:.0f} s")


def rows_10000_model64():
    """The float64 model of the 10^4 case's first 100 stored rows."""
    t0 = time.time()
    rows = np.loadtxt(os.path.join(HERE, "ellipsoids_10000_rows.txt"))[:100, 0].astype(np.int64)
    wl = W.ellipsoids_10000(W.STOKES)
    pr = O.Problem.from_workload(wl)
    cols = _model64_rows(pr, wl, rows, W.random_vector(pr.n_gamma, 87), W.smooth_vector(wl, 88))
    out = np.concatenate([rows[:, None].astype(np.float64)] + [c.reshape(-1, 3) for c in cols], axis=1)
    hdr = ("the float64 model (oracle/fp32_model.py, dt = float64) of the first 100 stored rows of "
           "ellipsoids_10000_rows.txt;\ncolumns: row, right-hand side b (3), A g (3), A s (3) (the same vectors).\n"
           f"{time.time() - t0:.0f} s.  Written by tests/golden/make_golden.py rows_10000_model64 (oracle/ only).")
    np.savetxt(os.path.join(HERE, "ellipsoids_10000_model64_rows.txt"), out, fmt="%.17e", header=hdr)
    _log("10^4 float64 model rows stored")


JOBS = {"grad_200": grad_200, "e100_tight": e100_tight, "rows_1000_model64": rows_1000_model64, "rows_10000_model64": rows_10000_model64, "rows_1000": rows_1000, "rows_10000_model": rows_10000_model, "two_way": two_way, "rows_10000": rows_10000, "batched": batched,
        "e1000_laplace": lambda: e1000(W.LAPLACE), "e1000_stokes": lambda: e1000(W.STOKES)}


def main():
    if len(sys.argv) == 1:
        return e100()
    for job in sys.argv[1:]:
        JOBS[job]()


if __name__ == "__main__":
    main()
