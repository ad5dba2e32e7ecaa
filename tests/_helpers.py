"""Shared test helpers: workload <-> device tensors, error norms."""
from __future__ import annotations

import numpy as np


def rel_inf(x, ref) -> float:
    """max |x - ref| / max |ref| over the whole stacked output."""
    x = np.asarray(x, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


def tight_reference(path):
    """A stored solution at GMRES tol 1e-13 (tests/golden/make_golden.py
    e100_tight) and, from its header, the final residual estimate rho of the
    oracle's solve at tol 1e-10 and that solve's output error err against it."""
    import re
    head = "".join(line for line in open(path) if line.startswith("#"))
    m = re.search(r"rho ([0-9.eE+-]+) err ([0-9.eE+-]+)", head)
    return np.loadtxt(path).reshape(-1), float(m.group(1)), float(m.group(2))


def structure(wl):
    """Host structure arrays of a workload: sys_body_ptr, body_trg_ptr, body_src_ptr."""
    n_trg = [wl.shapes[s].trg.shape[0] for s in wl.shape_of_body]
    n_src = [wl.shapes[s].src.shape[0] for s in wl.shape_of_body]
    return (np.asarray(wl.sys_body_ptr, np.int64), np.concatenate([[0], np.cumsum(n_trg)]).astype(np.int64),
            np.concatenate([[0], np.cumsum(n_src)]).astype(np.int64))


def net_flat(wl):
    return np.concatenate([np.asarray(n, np.float64).reshape(-1) for n in wl.net])


def stimson_jeffery_lambda(d: float, a: float = 1.0, terms: int = 400) -> float:
    """Exact drag factor of two equal spheres (radius a, centre distance d)
    translating with equal velocity U along their line of centres, from the
    bispherical-coordinate series of Stimson & Jeffery (Proc. R. Soc. A 111,
    1926; also Happel & Brenner, Low Reynolds Number Hydrodynamics, Sec. 6.3):
    the force on each sphere is 6 pi mu a U lambda with, for cosh(alpha) = d/(2a),

      lambda = (4/3) sinh(alpha) sum_{n>=1} n(n+1) / ((2n-1)(2n+3)) *
               [1 - (4 sinh^2((n+1/2) alpha) - (2n+1)^2 sinh^2(alpha))
                    / (2 sinh((2n+1) alpha) + (2n+1) sinh(2 alpha))].

    The terms fall like exp(-2 n alpha); 400 of them reach FP64 for gaps down
    to ~1e-3 a."""
    al = np.arccosh(d / (2.0 * a))
    s = 0.0
    for n in range(1, terms + 1):
        num = 4.0 * np.sinh((n + 0.5) * al) ** 2 - (2 * n + 1) ** 2 * np.sinh(al) ** 2
        den = 2.0 * np.sinh((2 * n + 1) * al) + (2 * n + 1) * np.sinh(2.0 * al)
        term = n * (n + 1) / ((2 * n - 1) * (2 * n + 3)) * (1.0 - num / den)
        s += term
        if n > 10 and abs(term) < 1e-18 * abs(s):
            break
    return 4.0 / 3.0 * np.sinh(al) * s


def two_sphere_workload(W, delta: float, n_src: int, n_trg: int, proxy_radius: float = 0.7):
    """Two unit spheres on the x axis, gap delta, equal unit forces along x."""
    shape = W.Shape(axes=np.ones(3), src=W.fibonacci_sphere(n_src, proxy_radius), trg=W.fibonacci_sphere(n_trg, 1.0))
    cen = np.array([[0.0, 0.0, 0.0], [2.0 + delta, 0.0, 0.0]])
    rot = np.repeat(np.eye(3)[None], 2, axis=0)
    net = np.array([[1.0, 0, 0, 0, 0, 0], [1.0, 0, 0, 0, 0, 0]])
    return W.Workload("two_spheres", [shape], cen, rot, np.zeros(2, np.int32), np.array([0, 2], np.int64),
                      np.array([W.STOKES], np.int32), [net])
