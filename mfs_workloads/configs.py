"""The five seeded synthetic workloads, as plain numpy arrays.

Each builder returns a ``Workload``: shapes (local proxy and collocation point
sets), bodies (centre, rotation, shape id), systems (body ranges and PDE kind)
and the given net quantities (charges q, or forces and torques F).  Nothing
here computes any part of the MFS method.

Recipes (the paper's own clusters and node files are not published):

* single_sphere   - one unit sphere, 600 Fibonacci collocation points at r=1,
                    300 Fibonacci proxies at r=0.7.  Stokes: f, t ~ N(0,1)^3;
                    Laplace: q = 1.
* ellipsoids_100  - 100 prolate spheroids (1,1,2) in a cube at volume
                    fraction 0.2 (side 16.12), uniform SO(3) orientations,
                    pairwise surface gap >= 0.1; M=800 collocation points on
                    the surface, N=400 proxies on the 0.7-scaled spheroid;
                    F, T ~ N(0,1).
* ellipsoids_1000 - as above with 1000 bodies (side 34.73); Stokes F, T and
                    Laplace q ~ N(0,1).
* batched_64      - 64 independent suspensions, body counts
                    floor(exp U(ln 10, ln 500)), systems 0-31 Stokes and
                    32-63 Laplace, one spheroid (1,1,r) with r ~ U[1,3] per
                    suspension, gap ~ U[0.05, 0.2] per suspension, volume
                    fraction 0.2, N=400, M=800.
* spheres_200     - 200 unit spheres, volume fraction 0.2 (side 16.12),
                    gap 0.1, N=400 proxies at r=0.7, M=800; F, T ~ N(0,1).

Seeds: workload i draws from ``np.random.default_rng(SeedSequence(1000+i))``
children: child 0 for the geometry, child 1 for the right-hand side.
"""
from __future__ import annotations

import dataclasses
import math
import os
from typing import List

import numpy as np

from .geometry import (compact_sphere_cluster, ellipsoid_ring_grid, fibonacci_sphere, fibonacci_spheroid, grown_sphere_cluster,
                       random_cluster, random_rotation, ring_grid_size, shift_inward)

LAPLACE = 0
STOKES = 1

PROXY_SCALE = 0.7
VOLUME_FRACTION = 0.2


@dataclasses.dataclass
class Shape:
    axes: np.ndarray          # (3,) semi-axes of the physical surface
    src: np.ndarray           # (N, 3) proxy points, body frame
    trg: np.ndarray           # (M, 3) collocation points, body frame


@dataclasses.dataclass
class Workload:
    name: str
    shapes: List[Shape]
    centre: np.ndarray        # (P, 3)
    rot: np.ndarray           # (P, 3, 3); world point = centre + rot @ local
    shape_of_body: np.ndarray # (P,) int32
    sys_body_ptr: np.ndarray  # (n_sys + 1,) int64, bodies of system s are [ptr[s], ptr[s+1])
    sys_kind: np.ndarray      # (n_sys,) int32, LAPLACE or STOKES
    net: List[np.ndarray]     # per system: (P_s,) charges or (P_s, 6) [f, t]
    mu: float = 1.0

    @property
    def n_body(self) -> int:
        return int(self.centre.shape[0])

    @property
    def n_sys(self) -> int:
        return int(self.sys_kind.shape[0])

    def world_points(self, which: str):
        """Stacked world coordinates and body ids of all proxies ('src') or
        collocation points ('trg'), bodies in order."""
        pts, ids = [], []
        for k in range(self.n_body):
            sh = self.shapes[self.shape_of_body[k]]
            loc = sh.src if which == "src" else sh.trg
            pts.append(self.centre[k] + loc @ self.rot[k].T)
            ids.append(np.full(loc.shape[0], k, dtype=np.int32))
        return np.concatenate(pts), np.concatenate(ids)

    def system(self, s: int) -> "Workload":
        """The single-system workload made of system s alone."""
        b0, b1 = int(self.sys_body_ptr[s]), int(self.sys_body_ptr[s + 1])
        used = sorted(set(int(x) for x in self.shape_of_body[b0:b1]))
        remap = {old: new for new, old in enumerate(used)}
        return Workload(
            name=f"{self.name}[{s}]",
            shapes=[self.shapes[i] for i in used],
            centre=self.centre[b0:b1].copy(),
            rot=self.rot[b0:b1].copy(),
            shape_of_body=np.array([remap[int(x)] for x in self.shape_of_body[b0:b1]], dtype=np.int32),
            sys_body_ptr=np.array([0, b1 - b0], dtype=np.int64),
            sys_kind=self.sys_kind[s:s + 1].copy(),
            net=[self.net[s].copy()],
            mu=self.mu,
        )


def _rngs(index: int):
    ss = np.random.SeedSequence(1000 + index)
    g, r = ss.spawn(2)
    return np.random.default_rng(g), np.random.default_rng(r)


def spheroid_shape(a: float, c: float, n_src: int, n_trg: int, scale: float = PROXY_SCALE) -> Shape:
    return Shape(axes=np.array([a, a, c], dtype=np.float64),
                 src=fibonacci_spheroid(n_src, scale * a, scale * c),
                 trg=fibonacci_spheroid(n_trg, a, c))


def cube_side(n_body: int, axes, fraction: float = VOLUME_FRACTION) -> float:
    return (n_body * (4.0 * math.pi / 3.0) * float(np.prod(axes)) / fraction) ** (1.0 / 3.0)


def single_sphere(kind: int = STOKES, n_src: int = 300, n_trg: int = 600,
                  radius: float = 1.0, proxy_radius: float = 0.7) -> Workload:
    """One sphere; Stokes F ~ N(0,1)^6 or Laplace q = 1."""
    _, rr = _rngs(0)
    shape = Shape(axes=np.full(3, radius), src=fibonacci_sphere(n_src, proxy_radius),
                  trg=fibonacci_sphere(n_trg, radius))
    net = rr.standard_normal((1, 6)) if kind == STOKES else np.ones(1)
    return Workload("single_sphere", [shape], np.zeros((1, 3)), np.eye(3)[None].copy(),
                    np.zeros(1, np.int32), np.array([0, 1], np.int64),
                    np.array([kind], np.int32), [net])


def _ellipsoid_suspension(index: int, n_body: int, kind: int, name: str,
                          n_src=400, n_trg=800, gap=0.1) -> Workload:
    rg, rr = _rngs(index)
    shape = spheroid_shape(1.0, 2.0, n_src, n_trg)
    box = cube_side(n_body, shape.axes)
    cen, rot = random_cluster(rg, n_body, shape.axes, box, gap)
    net = rr.standard_normal((n_body, 6)) if kind == STOKES else rr.standard_normal(n_body)
    return Workload(name, [shape], cen, rot, np.zeros(n_body, np.int32),
                    np.array([0, n_body], np.int64), np.array([kind], np.int32), [net])


def ellipsoids_100(kind: int = STOKES) -> Workload:
    return _ellipsoid_suspension(1, 100, kind, "ellipsoids_100")


def ellipsoids_1000(kind: int = STOKES) -> Workload:
    return _cached(f"ellipsoids_1000_k{kind}", lambda: _ellipsoid_suspension(2, 1000, kind, "ellipsoids_1000"))


_CACHE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_cache")


def _cached(key: str, make):
    """Geometry generation for 1000 ellipsoids takes tens of seconds in Python;
    keep the arrays in an untracked .npz beside this module (regenerated when
    missing, identical either way since the draw is seeded)."""
    path = os.path.join(_CACHE_DIR, key + ".npz")
    if os.path.exists(path):
        try:
            z = np.load(path, allow_pickle=False)
            shapes = [Shape(z[f"ax{i}"], z[f"src{i}"], z[f"trg{i}"]) for i in range(int(z["n_shape"]))]
            nets = [z[f"net{i}"] for i in range(int(z["n_sys"]))]
            return Workload(str(z["name"]), shapes, z["centre"], z["rot"], z["shape_of_body"],
                            z["sys_body_ptr"], z["sys_kind"], nets, float(z["mu"]))
        except Exception:
            pass
    w = make()
    try:
        os.makedirs(_CACHE_DIR, exist_ok=True)
        arrs = dict(name=np.array(w.name), n_shape=np.array(len(w.shapes)), n_sys=np.array(w.n_sys),
                    centre=w.centre, rot=w.rot, shape_of_body=w.shape_of_body,
                    sys_body_ptr=w.sys_body_ptr, sys_kind=w.sys_kind, mu=np.array(w.mu))
        for i, sh in enumerate(w.shapes):
            arrs[f"ax{i}"], arrs[f"src{i}"], arrs[f"trg{i}"] = sh.axes, sh.src, sh.trg
        for i, n in enumerate(w.net):
            arrs[f"net{i}"] = n
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, **arrs)
        os.replace(tmp, path)
    except OSError:
        pass
    return w


def batched_64(n_sys: int = 64, n_src: int = 400, n_trg: int = 800, p_min=10, p_max=500) -> Workload:
    if (n_sys, n_src, n_trg, p_min, p_max) == (64, 400, 800, 10, 500):
        return _cached("batched_64", lambda: _batched(n_sys, n_src, n_trg, p_min, p_max))
    return _batched(n_sys, n_src, n_trg, p_min, p_max)


def _batched(n_sys, n_src, n_trg, p_min, p_max) -> Workload:
    rg, rr = _rngs(3)
    shapes, cens, rots, sob, ptr, kinds, nets = [], [], [], [], [0], [], []
    for s in range(n_sys):
        p = int(math.floor(math.exp(rg.uniform(math.log(p_min), math.log(p_max)))))
        r = rg.uniform(1.0, 3.0)
        gap = rg.uniform(0.05, 0.2)
        kind = STOKES if s < n_sys // 2 else LAPLACE
        shape = spheroid_shape(1.0, r, n_src, n_trg)
        box = cube_side(p, shape.axes)
        cen, rot = random_cluster(rg, p, shape.axes, box, gap)
        shapes.append(shape)
        cens.append(cen)
        rots.append(rot)
        sob.append(np.full(p, s, np.int32))
        ptr.append(ptr[-1] + p)
        kinds.append(kind)
        nets.append(rr.standard_normal((p, 6)) if kind == STOKES else rr.standard_normal(p))
    return Workload("batched_64", shapes, np.concatenate(cens), np.concatenate(rots),
                    np.concatenate(sob), np.array(ptr, np.int64), np.array(kinds, np.int32), nets)


def spheres_200(n_body: int = 200, n_src=400, n_trg=800, gap=0.1) -> Workload:
    rg, rr = _rngs(4)
    shape = Shape(axes=np.ones(3), src=fibonacci_sphere(n_src, PROXY_SCALE), trg=fibonacci_sphere(n_trg, 1.0))
    box = cube_side(n_body, shape.axes)
    cen, rot = random_cluster(rg, n_body, shape.axes, box, gap)
    net = rr.standard_normal((n_body, 6))
    return Workload("spheres_200", [shape], cen, rot, np.zeros(n_body, np.int32),
                    np.array([0, n_body], np.int64), np.array([STOKES], np.int32), [net])


def small_cluster(n_body: int, kind: int, n_src: int, n_trg: int, seed: int, axes=(1.0, 1.0, 2.0),
                  gap: float = 0.1, fraction: float = VOLUME_FRACTION) -> Workload:
    """A small random cluster for parity tests (sizes the oracle finishes in seconds)."""
    ss = np.random.SeedSequence(5000 + seed)
    g, r = ss.spawn(2)
    rg, rr = np.random.default_rng(g), np.random.default_rng(r)
    shape = spheroid_shape(axes[0], axes[2], n_src, n_trg)
    box = cube_side(n_body, shape.axes, fraction)
    cen, rot = random_cluster(rg, n_body, shape.axes, box, gap)
    net = rr.standard_normal((n_body, 6)) if kind == STOKES else rr.standard_normal(n_body)
    return Workload(f"small_{n_body}_{kind}_{seed}", [shape], cen, rot, np.zeros(n_body, np.int32),
                    np.array([0, n_body], np.int64), np.array([kind], np.int32), [net])


TYPE_T_AXES = (0.4, 0.6, 1.0)
DELTA_SEP_MOBILITY = 1.05 * 0.125


def type_t_shape(n_v: int = 34, delta_sep: float = DELTA_SEP_MOBILITY) -> Shape:
    """The paper's Type T triaxial ellipsoid (semi-axes 0.4, 0.6, 1) on its
    ring grid (Section 4.2): proxies on the n_v-ring grid moved inward by
    delta_sep along the normal; collocation points on the grid with 1.15 n_v
    Gauss-Legendre rings.  n_v = 34 gives N = 658, M = 842."""
    axes = np.array(TYPE_T_AXES, dtype=np.float64)
    trg = ellipsoid_ring_grid(*TYPE_T_AXES, int(round(1.15 * n_v)), n_total=ring_grid_size(1.15 * n_v))
    src = shift_inward(ellipsoid_ring_grid(*TYPE_T_AXES, n_v), axes, delta_sep)
    return Shape(axes=axes, src=src, trg=trg)


def _type_t_cluster(rg, rr, n_body: int, kind: int, delta: float, n_v: int, name: str) -> Workload:
    cen = grown_sphere_cluster(rg, n_body, delta)
    rot = np.stack([random_rotation(rg) for _ in range(n_body)])
    net = rr.standard_normal((n_body, 6)) if kind == STOKES else rr.standard_normal(n_body)
    return Workload(name, [type_t_shape(n_v)], cen, rot, np.zeros(n_body, np.int32),
                    np.array([0, n_body], np.int64), np.array([kind], np.int32), [net])


def ellipsoids_10000(kind: int = STOKES) -> Workload:
    """The paper's large demonstration (Section 4.2): 10^4 Type T ellipsoids,
    each inside one sphere of a grown unit-sphere cluster whose spheres are
    delta = 0.2 from at least one neighbour, orientations uniform on SO(3);
    N = 658, M = 842 (n_v = 34); forces and torques (or charges) N(0,1)."""
    def make():
        rg, rr = _rngs(5)
        return _type_t_cluster(rg, rr, 10000, kind, 0.2, 34, "ellipsoids_10000")
    return _cached(f"ellipsoids_10000_k{kind}", make)


def type_t_cluster(n_body: int, kind: int, seed: int, delta: float = 0.2, n_v: int = 34) -> Workload:
    """A smaller cluster built like ellipsoids_10000 (for parity tests)."""
    g, r = np.random.SeedSequence(5000 + seed).spawn(2)
    return _type_t_cluster(np.random.default_rng(g), np.random.default_rng(r), n_body, kind, delta, n_v,
                           f"type_t_{n_body}_{kind}_{seed}")


def surface_test_points(shape: Shape, n: int = 1732) -> np.ndarray:
    """n points on the physical surface of a shape (body frame) for the surface
    residual; the paper uses 1732 per particle (Section 4.2).  Spheroids: the
    equal-area Fibonacci lattice; other ellipsoids: the ring grid with n nodes."""
    a, b, c = (float(x) for x in shape.axes)
    if abs(a - b) < 1e-15:
        return fibonacci_spheroid(n, a, c)
    n_v = int(round((-3.9 + math.sqrt(3.9 ** 2 + 4 * 0.44 * (n - 17))) / (2 * 0.44)))
    return ellipsoid_ring_grid(a, b, c, n_v, n_total=n)


def with_proxy_scale(wl: Workload, scale: float) -> Workload:
    """The same suspension with every shape's proxies regenerated on the
    surface scaled by `scale` (same count).  For the 2-way error, which pairs
    two formulations on distinct proxy surfaces."""
    shapes = []
    for sh in wl.shapes:
        a, b, c = (float(x) for x in sh.axes)
        assert abs(a - b) < 1e-15, "proxy regeneration supports spheroids (a, a, c)"
        shapes.append(Shape(axes=sh.axes.copy(), src=fibonacci_spheroid(sh.src.shape[0], scale * a, scale * c),
                            trg=sh.trg.copy()))
    return dataclasses.replace(wl, name=f"{wl.name}@proxy{scale:.4f}", shapes=shapes)


def resistance_proxy_scale(mobility_scale: float = PROXY_SCALE) -> float:
    """Proxy scale of the resistance problem paired with a mobility problem
    for the 2-way error: Delta_sep^mob = 1.05 Delta_sep^res (Section 4), with
    Delta_sep = 1 - scale."""
    return 1.0 - (1.0 - mobility_scale) / 1.05


def random_vector(n: int, seed: int) -> np.ndarray:
    """A seeded N(0,1) vector (matvec inputs for parity tests)."""
    return np.random.default_rng(np.random.SeedSequence(9000 + seed)).standard_normal(n)


def smooth_vector(wl: Workload, seed: int) -> np.ndarray:
    """A seeded smooth field on the collocation points (gamma layout): per body,
    a random polynomial of degree 2 in the body-frame coordinates (a vector
    polynomial for Stokes systems, scalar for Laplace).  Stands in for the
    smooth surface data GMRES works with."""
    rng = np.random.default_rng(np.random.SeedSequence(9500 + seed))
    parts = []
    for s in range(wl.n_sys):
        dim = 3 if wl.sys_kind[s] == STOKES else 1
        for b in range(int(wl.sys_body_ptr[s]), int(wl.sys_body_ptr[s + 1])):
            x = wl.shapes[wl.shape_of_body[b]].trg
            feats = np.concatenate([np.ones((x.shape[0], 1)), x, x * x, x[:, [0]] * x[:, [1]],
                                    x[:, [1]] * x[:, [2]], x[:, [0]] * x[:, [2]]], axis=1)
            coef = rng.standard_normal((feats.shape[1], dim))
            parts.append((feats @ coef).reshape(-1))
    return np.concatenate(parts)


def elastance_spheres(n_src: int = 969, n_trg: int = 1123, n_body: int = 10, delta: float = 0.1,
                      seed: int = 0) -> Workload:
    """The paper's small elastance test (Section 4.1): n_body unit spheres grown
    compactly from the origin at minimum gap delta (compact_sphere_cluster),
    N proxies on the concentric sphere of radius R_p = 0.7 and M collocation
    points on the surface (N = 969, M = 1123 as in the paper), Fibonacci point
    sets in place of its spherical designs.  Net charges q ~ N(0, 1) (the paper
    does not state them)."""
    g, r = np.random.SeedSequence(7000 + seed).spawn(2)
    cen = compact_sphere_cluster(np.random.default_rng(g), n_body, delta)
    q = np.random.default_rng(r).standard_normal(n_body)
    shape = Shape(axes=np.ones(3), src=fibonacci_sphere(n_src, PROXY_SCALE), trg=fibonacci_sphere(n_trg, 1.0))
    rot = np.repeat(np.eye(3)[None], n_body, axis=0)
    return Workload("elastance_spheres", [shape], cen, rot, np.zeros(n_body, np.int32),
                    np.array([0, n_body], np.int64), np.array([LAPLACE], np.int32), [q])
