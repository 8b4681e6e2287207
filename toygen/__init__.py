"""Seeded synthetic inputs (detector descriptions, tracks, hits, noise pools).

Shared by the tests, the benchmark and the smoke check.  It holds no part of
the Kalman filter itself: only the toy physics that produces inputs.
"""
from .detector import BARREL, DISK, Geometry, Workload, workloads, barrel_geometry, mixed_geometry, geometric_radii
from .candidates import duplicate_candidates
from .generate import Event, HitPools, generate, make_pools, subset, truncate, with_modules
from .tilted import ModuleGeometry, PlaneEvent, PlaneWorkload, generate_planes, plane_workloads, tilted_barrel

__all__ = ["BARREL", "DISK", "Geometry", "Workload", "workloads", "barrel_geometry", "mixed_geometry",
           "geometric_radii", "Event", "HitPools", "generate", "make_pools", "subset", "truncate", "with_modules",
           "duplicate_candidates", "ModuleGeometry", "PlaneEvent", "PlaneWorkload", "generate_planes",
           "plane_workloads", "tilted_barrel"]
