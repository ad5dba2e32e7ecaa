"""Writes the oracle's solutions of the 100-ellipsoid workload (FP64, GMRES
tol 1e-10) to text files next to this script.  Calls only oracle/ and the
seeded input generators; takes a few minutes on 8 cores.

    python tests/golden/make_golden.py
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


def main():
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
