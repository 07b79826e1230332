"""Seeded synthetic inputs (meshes, noise) shared by the oracle and the GPU library.

Holds none of the method's arithmetic; see ``meshes`` for the generators.
"""
from .meshes import (Mesh, kuhn_cube, notched_cube, hull_mesh, radius_ratio, workload_mesh,
                     WORKLOADS, sphere_points, ellipsoid_points, morton_renumber,
                     kuhn_square, polygon_mesh, circle_points, fibonacci_sphere)

__all__ = ["Mesh", "kuhn_cube", "notched_cube", "hull_mesh", "radius_ratio", "workload_mesh",
           "WORKLOADS", "sphere_points", "ellipsoid_points", "morton_renumber",
           "kuhn_square", "polygon_mesh", "circle_points", "fibonacci_sphere"]
