"""Writes the oracle's solutions of the 100-ellipsoid workload (FP64, GMRES
tol 1e-10) to text files next to this script.  Calls only oracle/ and the
seeded input generators; takes a few minutes on 8 cores.

    python tests/golden/make_golden.py            # mobility / elastance solutions
    python tests/golden/make_golden.py two_way    # resistance -> mobility (2-way error)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mfs_workloads as W  # noqa: E402
from oracle import mfs_oracle as O  # noqa: E402


def two_way():
    """Resistance solve of ellipsoids_100 (proxies at the resistance scale) with
    seeded rigid velocities U_ref, then the mobility solve (proxies at 0.7)
    with the resulting forces: stores U_ref, F and U (eq. (2way))."""
    wl = W.ellipsoids_100(W.STOKES)
    wr = W.with_proxy_scale(wl, W.resistance_proxy_scale())
    U_ref = np.random.default_rng(np.random.SeedSequence(7100)).standard_normal((wl.n_body, 6))
    t0 = time.time()
    r = O.two_way_error(O.ResistanceProblem.from_workload(wr), O.Problem.from_workload(wl), U_ref, tol=1e-10)
    dt = time.time() - t0
    hdr = (f"2-way test of the seeded ellipsoids_100 workload: columns U_ref (6), F (6), U (6) per body;\n"
           f"resistance proxies at scale {W.resistance_proxy_scale():.6f}, mobility at 0.7; U_ref from "
           f"SeedSequence(7100); FP64 oracle, GMRES tol 1e-10,\n"
           f"{r['iters_res']} resistance + {r['iters_mob']} mobility iterations, {dt:.0f} s; eps_2way = "
           f"{r['eps']:.6e}.  Written by tests/golden/make_golden.py two_way (oracle only).")
    np.savetxt(os.path.join(HERE, "ellipsoids_100_two_way.txt"),
               np.concatenate([U_ref, r["F"].reshape(-1, 6), r["U"].reshape(-1, 6)], axis=1), fmt="%.17e", header=hdr)
    print("two_way", r["iters_res"], r["iters_mob"], r["eps"], f"{dt:.0f}s", flush=True)


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "two_way":
        return two_way()
    for kind, name, what in ((W.STOKES, "ellipsoids_100_stokes_U.txt", "rigid velocities [v; omega] per body"),
                             (W.LAPLACE, "ellipsoids_100_laplace_phi.txt", "potentials per body")):
        wl = W.ellipsoids_100(kind)
        t0 = time.time()
        sol = O.Problem.from_workload(wl).solve(wl.net[0], tol=1e-10)
        dt = time.time() - t0
        out = np.asarray(sol["out"]).reshape(wl.n_body, -1)
        hdr = (f"oracle solution of the seeded ellipsoids_100 workload ({'Stokes mobility' if kind else 'Laplace elastance'}),\n"
               f"{what}; FP64 oracle, GMRES tol 1e-10, {sol['iters']} iterations, {dt:.0f} s.\n"
               f"Written by tests/golden/make_golden.py (oracle only).")
        np.savetxt(os.path.join(HERE, name), out, fmt="%.17e", header=hdr)
        print(name, sol["iters"], f"{dt:.0f}s", flush=True)


if __name__ == "__main__":
    main()
