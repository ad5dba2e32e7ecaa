"""Seeded synthetic geometry: point sets on spheroids and random particle clusters.

This module generates *inputs* only.  It holds none of the MFS arithmetic
(no kernels, no projections, no solves); both the oracle and the GPU path
read the arrays it returns.

Point sets
----------
The paper discretises spheres with spherical designs and ellipsoids with a
Gauss-Legendre / trapezoidal grid (Section 4.1 and Section 4.2).  Neither
node file ships with the paper, so the stand-in is a Fibonacci lattice:
z_i = 1 - (2i+1)/n, azimuth theta_i = i*pi*(3 - sqrt 5).  For a spheroid with
semi-axes (a, a, c) the height of node i is instead placed at the equal-area
quantile (i + 1/2)/n of the spheroid's surface (measured from the top), so the
lattice stays quasi-uniform in area, as the paper asks of its node sets.

Clusters
--------
Centres are uniform in a cube [0, L]^3, orientations uniform on SO(3)
(normalised Gaussian quaternion), and candidates are rejected until every pair
of bodies is at least a given surface gap apart.  The exact surface distance
between two ellipsoids is found by alternating projection between the two
solid ellipsoids (the paper uses the same device to measure separations,
Section 4.2).  Alternating projection decreases the distance estimate
monotonically towards the true distance, so a candidate is rejected as soon
as the estimate falls below the gap and accepted only once it has converged.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = math.pi * (3.0 - math.sqrt(5.0))


def fibonacci_sphere(n: int, radius: float = 1.0) -> np.ndarray:
    """n quasi-uniform points on the sphere of the given radius, shape (n, 3)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = i * GOLDEN
    return radius * np.stack([rho * np.cos(th), rho * np.sin(th), z], axis=1)


def _spheroid_height_quantiles(n: int, a: float, c: float) -> np.ndarray:
    """Heights z in [-c, c] that split the spheroid (a, a, c) surface into n
    equal-area bands (node i at the centre of band i, counted from the top)."""
    if abs(a - c) < 1e-15:
        i = np.arange(n, dtype=np.float64)
        return c * (1.0 - (2.0 * i + 1.0) / n)
    # Surface of revolution with radius rho(z) = a sqrt(1 - z^2/c^2).  Its area
    # element per unit t = z/c is 2 pi a c sqrt(1 - e t^2) with e = 1 - a^2/c^2.
    t = np.linspace(-1.0, 1.0, 200001)
    e = 1.0 - (a * a) / (c * c)
    dens = np.sqrt(np.maximum(0.0, 1.0 - e * t * t))
    cum = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(t))])
    cum /= cum[-1]
    i = np.arange(n, dtype=np.float64)
    frac_from_top = (i + 0.5) / n
    tq = np.interp(1.0 - frac_from_top, cum, t)
    return c * tq


def fibonacci_spheroid(n: int, a: float, c: float) -> np.ndarray:
    """n quasi-uniform points on the spheroid x^2/a^2 + y^2/a^2 + z^2/c^2 = 1."""
    z = _spheroid_height_quantiles(n, a, c)
    rho = a * np.sqrt(np.maximum(0.0, 1.0 - (z / c) ** 2))
    th = np.arange(n, dtype=np.float64) * GOLDEN
    return np.stack([rho * np.cos(th), rho * np.sin(th), z], axis=1)


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3) from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _project_solid_ellipsoid(q: np.ndarray, axes: np.ndarray) -> np.ndarray:
    """Closest point to q (local frame) of the solid ellipsoid with the given semi-axes."""
    if np.sum((q / axes) ** 2) <= 1.0:
        return q.copy()
    a2 = axes * axes
    t = 0.0
    for _ in range(100):
        den = a2 + t
        f = np.sum(a2 * q * q / (den * den)) - 1.0
        fp = -2.0 * np.sum(a2 * q * q / (den * den * den))
        step = f / fp
        t -= step
        if abs(step) <= 1e-15 * max(1.0, t):
            break
    return a2 * q / (a2 + t)


def ellipsoid_gap_at_least(c1, R1, ax1, c2, R2, ax2, gap, max_iter=400) -> bool:
    """True iff the surface distance between the two solid ellipsoids is >= gap.

    Ellipsoid k is {c_k + R_k z : sum(z_i^2/ax_k,i^2) <= 1}."""
    dc = np.linalg.norm(c2 - c1)
    if dc >= ax1.max() + ax2.max() + gap:
        return True
    if dc < ax1.min() + ax2.min() + gap:
        return False
    p2 = c2.copy()
    prev = np.inf
    for _ in range(max_iter):
        p1 = c1 + R1 @ _project_solid_ellipsoid(R1.T @ (p2 - c1), ax1)
        p2 = c2 + R2 @ _project_solid_ellipsoid(R2.T @ (p1 - c2), ax2)
        d = np.linalg.norm(p2 - p1)
        if d < gap:
            return False
        if prev - d <= 1e-12 * max(1.0, d):
            return True
        prev = d
    return True


def random_cluster(rng: np.random.Generator, n_body: int, axes, box: float, gap: float,
                   max_tries: int = 2_000_000):
    """Random sequential addition of n_body ellipsoids of the given semi-axes
    (one (3,) array, or an (n_body, 3) array) in the cube [0, box]^3 with
    pairwise surface gap >= gap.  Returns (centres (P,3), rotations (P,3,3))."""
    axes = np.asarray(axes, dtype=np.float64)
    if axes.ndim == 1:
        axes = np.broadcast_to(axes, (n_body, 3)).copy()
    spherical = np.all(np.abs(axes - axes[:, :1]) == 0.0, axis=1)
    rmax = axes.max(axis=1)
    cell = 2.0 * rmax.max() + gap
    ncell = max(1, int(box // cell))
    grid: dict = {}
    cen = np.zeros((n_body, 3))
    rot = np.zeros((n_body, 3, 3))
    k = 0
    tries = 0
    while k < n_body:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("random_cluster: could not place all bodies")
        c = rng.uniform(0.0, box, size=3)
        R = random_rotation(rng)
        key = tuple(np.minimum((c / cell).astype(int), ncell - 1))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if spherical[k] and spherical[j]:
                            ok = np.linalg.norm(cen[j] - c) >= axes[k, 0] + axes[j, 0] + gap
                        else:
                            ok = ellipsoid_gap_at_least(cen[j], rot[j], axes[j], c, R, axes[k], gap)
                        if not ok:
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        cen[k] = c
        rot[k] = R
        grid.setdefault(key, []).append(k)
        k += 1
    return cen, rot


# ---------------------------------------------------------------------------
# The paper's large-cluster geometry (Section 4.2)
# ---------------------------------------------------------------------------

def _ellipse_perimeter(p: float, q: float) -> float:
    """Perimeter of the ellipse with semi-axes p, q (Ramanujan's second formula)."""
    if p + q == 0.0:
        return 0.0
    h = ((p - q) / (p + q)) ** 2
    return math.pi * (p + q) * (1.0 + 3.0 * h / (10.0 + math.sqrt(4.0 - 3.0 * h)))


def ring_grid_size(n_v: float) -> int:
    """The paper's node count of its ellipsoid grid, 17 + 3.9 n_v + 0.44 n_v^2 (Section 4.2)."""
    return int(round(17.0 + 3.9 * n_v + 0.44 * n_v * n_v))


def ellipsoid_ring_grid(a: float, b: float, c: float, n_v: int, n_total: int = 0) -> np.ndarray:
    """Quasi-uniform grid on the ellipsoid x^2/a^2 + y^2/b^2 + z^2/c^2 = 1 as the
    paper describes it (Section 4.2): parameterise the surface by
    (a sqrt(1-t^2) cos s, b sqrt(1-t^2) sin s, c t), take n_v Gauss-Legendre
    nodes in t and, on each ring, equispaced (trapezoidal) nodes in s whose
    count is proportional to the ring's perimeter (at least 3).  The
    proportionality constant is chosen so the total is as close as possible to
    n_total (default: the paper's count for n_v, ring_grid_size).  Consecutive
    rings are rotated by half a step.  Returns (n, 3)."""
    t, _ = np.polynomial.legendre.leggauss(n_v)
    rho = np.sqrt(1.0 - t * t)
    per = np.array([_ellipse_perimeter(a * r, b * r) for r in rho])
    target = n_total or ring_grid_size(n_v)

    def counts_for(k):
        return np.maximum(3, np.rint(k * per / per.max()).astype(int))

    lo, hi = 1.0, 4.0 * n_v
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if counts_for(mid).sum() < target:
            lo = mid
        else:
            hi = mid
    counts = min((counts_for(lo), counts_for(hi)), key=lambda q: abs(int(q.sum()) - target))
    pts = []
    for i, (ti, ri, ni) in enumerate(zip(t, rho, counts)):
        s = 2.0 * math.pi * (np.arange(ni) + 0.5 * (i % 2)) / ni
        pts.append(np.stack([a * ri * np.cos(s), b * ri * np.sin(s), np.full(ni, c * ti)], axis=1))
    return np.concatenate(pts)


def shift_inward(points: np.ndarray, axes, delta: float) -> np.ndarray:
    """Points on the ellipsoid surface moved a distance delta along the inward
    unit normal (the paper's normal-shifted proxy surface, Section 4.2)."""
    axes = np.asarray(axes, np.float64)
    n = points / (axes * axes)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return points - delta * n


def grown_sphere_cluster(rng: np.random.Generator, n: int, delta: float, radius: float = 1.0,
                         max_tries: int = 50_000_000) -> np.ndarray:
    """Centres of n spheres of the given radius, each exactly delta (surface
    gap) from at least one sphere placed before it and at least delta from all
    others: every new sphere is put at distance 2 radius + delta from a
    uniformly chosen earlier sphere in a uniform random direction, and kept if
    it clears all others (cell-list check).  The paper grows its 10^4-ellipsoid
    cluster from such a sphere cluster (Section 4.2)."""
    d = 2.0 * radius + delta
    cen = np.zeros((n, 3))
    grid: dict = {(0, 0, 0): [0]}
    k, tries = 1, 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("grown_sphere_cluster: could not place all spheres")
        u = rng.standard_normal(3)
        c = cen[rng.integers(k)] + d * u / np.linalg.norm(u)
        key = tuple(np.floor(c / d).astype(int))
        ok = True
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for j in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if np.sum((cen[j] - c) ** 2) < d * d * (1.0 - 1e-12):
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        cen[k] = c
        grid.setdefault(key, []).append(k)
        k += 1
    return cen

def compact_sphere_cluster(rng: np.random.Generator, n: int, delta: float, radius: float = 1.0) -> np.ndarray:
    """Centres of n spheres grown from the origin as in the paper's small
    elastance test (Section 4.1): the first sphere sits at the origin; each new one
    is placed along a uniformly random direction u at the smallest distance t
    from the origin where its surface gap to every placed sphere is at least
    delta, so the gap to at least one of them is exactly delta.  For a placed
    centre p the forbidden distances are the roots interval of
    |t u - p|^2 < (2 radius + delta)^2; t is the smallest t >= 0 outside all of
    them."""
    d = 2.0 * radius + delta
    cen = np.zeros((n, 3))
    for k in range(1, n):
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        b = cen[:k] @ u
        disc = b * b - (np.sum(cen[:k] ** 2, axis=1) - d * d)
        iv = sorted((bi - np.sqrt(di), bi + np.sqrt(di)) for bi, di in zip(b, disc) if di > 0.0)
        t = 0.0
        for lo, hi in iv:  # sweep the forbidden intervals in order of their start
            if lo <= t < hi:
                t = hi
        cen[k] = t * u
    return cen
