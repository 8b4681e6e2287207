"""Toy detector descriptions and workload recipes.

A *layer* follows the paper's definition (Sec. 3.1, "Geometry & detector
description"): an r-z bounding box in global cylindrical coordinates.  Here it
is either a barrel cylinder r = R with z in [lo, hi] or an endcap disk z = Z
with r in [lo, hi].  Each layer also carries its material thickness in
radiation lengths at normal incidence (the paper extracts material per layer,
same section).

This module holds only descriptions and sizes; no part of the Kalman filter.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BARREL = 0
DISK = 1

# Radii (cm) of the ten-cylinder barrel.
BARREL10_RADII = (4.0, 7.0, 11.0, 16.0, 25.0, 35.0, 50.0, 65.0, 85.0, 110.0)
BARREL_HALF_LENGTH = 150.0
MATERIAL_X_OVER_X0 = 0.02


def geometric_radii(n: int = 20, r_min: float = 4.0, r_max: float = 110.0) -> np.ndarray:
    """n radii spaced geometrically between r_min and r_max (inclusive)."""
    i = np.arange(n, dtype=np.float64)
    return r_min * (r_max / r_min) ** (i / (n - 1))


def disk_positions(n_per_side: int = 8, z_min: float = 30.0, z_max: float = 270.0) -> np.ndarray:
    k = np.arange(n_per_side, dtype=np.float64)
    return z_min + (z_max - z_min) * k / (n_per_side - 1)


@dataclass(frozen=True)
class Geometry:
    kind: np.ndarray        # int8 [L]: 0 barrel, 1 disk
    pos: np.ndarray         # float64 [L]: R (barrel) or Z (disk), cm
    lo: np.ndarray          # float64 [L]: zmin (barrel) or rmin (disk)
    hi: np.ndarray          # float64 [L]: zmax (barrel) or rmax (disk)
    x_over_x0: np.ndarray   # float64 [L]
    bz: float = 3.8         # tesla
    mass: float = 0.13957   # GeV, charged pion hypothesis

    @property
    def n_layers(self) -> int:
        return int(self.kind.shape[0])


def barrel_geometry(radii, half_length: float = BARREL_HALF_LENGTH,
                    x_over_x0: float = MATERIAL_X_OVER_X0, bz: float = 3.8) -> Geometry:
    r = np.asarray(radii, dtype=np.float64)
    n = r.shape[0]
    return Geometry(kind=np.zeros(n, np.int8), pos=r,
                    lo=np.full(n, -half_length), hi=np.full(n, half_length),
                    x_over_x0=np.full(n, x_over_x0), bz=bz)


def mixed_geometry(x_over_x0: float = MATERIAL_X_OVER_X0, bz: float = 3.8) -> Geometry:
    """Ten barrel cylinders plus eight disks on each side (+z first, then -z)."""
    rb = np.asarray(BARREL10_RADII)
    zd = disk_positions()
    kind = np.concatenate([np.zeros(10, np.int8), np.ones(16, np.int8)])
    pos = np.concatenate([rb, zd, -zd])
    lo = np.concatenate([np.full(10, -BARREL_HALF_LENGTH), np.full(16, 4.0)])
    hi = np.concatenate([np.full(10, BARREL_HALF_LENGTH), np.full(16, 110.0)])
    return Geometry(kind=kind, pos=pos, lo=lo, hi=hi,
                    x_over_x0=np.full(26, x_over_x0), bz=bz)


@dataclass(frozen=True)
class Workload:
    name: str
    geometry: Geometry
    n_tracks: int
    seed: int
    eta_max: float = 1.0
    pt_min: float = 0.5
    pt_max: float = 10.0
    mode: str = "outward"       # "outward": next barrel only; "nearest": any surface by path
    max_entries: int = 26
    hole_fraction: float = 0.0
    sigma_rphi: float = 0.003
    sigma_z: float = 0.01       # barrel z resolution
    sigma_r: float = 0.01       # disk r resolution
    sigma_n: float = 0.03 / np.sqrt(12.0)   # sensor-thickness term along the surface normal
    misalign_rphi: float = 0.0  # sigma of per-layer true offsets (cm)
    misalign_z: float = 0.0
    noise_density: float = 0.0  # noise hits per cm^2 of barrel surface
    stop_fraction: float = 0.0  # central tracks that end early (an interaction), after 3 .. n of their n crossings
    extra: dict = field(default_factory=dict)


def workloads() -> dict[str, Workload]:
    g10 = barrel_geometry(BARREL10_RADII)
    g20 = barrel_geometry(geometric_radii(20))
    return {
        # plain FP64 fit, ten barrel cylinders
        "barrel10": Workload("barrel10", g10, 1_000, 1001),
        # batched FP32 / FP64 fit, twenty geometric barrel layers
        "barrel20": Workload("barrel20", g20, 100_000, 1002),
        # uneven lengths: barrel + endcaps, loopers, 5% holes
        "mixed26": Workload("mixed26", mixed_geometry(), 500_000, 1003, eta_max=2.5,
                            mode="nearest", hole_fraction=0.05, stop_fraction=0.25),
        # combinatorial hit scoring with noise
        "search20": Workload("search20", g20, 20_000, 1004, noise_density=2.0),
        # adjoint with injected misalignment
        "align20": Workload("align20", g20, 100_000, 1005, misalign_rphi=0.005, misalign_z=0.01),
    }
