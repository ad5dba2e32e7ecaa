"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds geometry and right-hand-side generators only; no part of the MFS
method is computed here."""
from .configs import (LAPLACE, STOKES, Shape, Workload, batched_64, cube_side, ellipsoids_100, smooth_vector,
                      ellipsoids_1000, random_vector, resistance_proxy_scale, single_sphere, small_cluster,
                      spheres_200, spheroid_shape, with_proxy_scale, ellipsoids_10000, type_t_cluster, type_t_shape,
                      surface_test_points, elastance_spheres)
from .geometry import compact_sphere_cluster, fibonacci_sphere, fibonacci_spheroid, random_cluster, random_rotation

__all__ = [
    "LAPLACE", "STOKES", "Shape", "Workload", "batched_64", "cube_side", "ellipsoids_100",
    "ellipsoids_1000", "random_vector", "single_sphere", "small_cluster", "spheres_200",
    "spheroid_shape", "smooth_vector", "with_proxy_scale", "resistance_proxy_scale",
    "ellipsoids_10000", "type_t_cluster", "type_t_shape", "surface_test_points", "fibonacci_sphere", "fibonacci_spheroid", "random_cluster", "random_rotation",
    "elastance_spheres", "compact_sphere_cluster",
]
