"""The five scan configurations the project is measured on, as seeded inputs.

Sizes are in voxels; source-object (SOD) and source-detector (SDD) distances
are in voxel units, detector pitch in voxel units per pixel.  Where the
configuration leaves a constant open, the values below keep the tiny case's
proportions: SOD = 3.125 N, SDD = 2 SOD, pitch 1.5.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import phantoms, trajectories


@dataclass
class ScanConfig:
    name: str
    shape: tuple            # (nz, ny, nx)
    n_proj: int
    n_u: int
    n_v: int
    n_sub: int
    step: float
    P: np.ndarray           # [n_proj][n_sub][3][4] float64
    U: np.ndarray = None    # [g][g][g][3] float32 displacement grid, or None
    tau: np.ndarray = None  # [n_proj][n_sub] float64 time fractions, or None
    extra: dict = field(default_factory=dict)

    @property
    def n_voxels(self):
        return int(np.prod(self.shape))

    @property
    def n_rays(self):
        return self.n_proj * self.n_u * self.n_v


CONFIGS = ("tiny", "full", "helical", "diff", "learned")

SEED_BASE = 0


def make_config(name, n_proj=None, seed=SEED_BASE):
    """Geometry (and motion) of a named configuration.

    ``n_proj`` overrides the projection count (test subsets keep the angular
    spacing of the full scan only when they pick views from the full list).
    """
    if name == "tiny":
        N = 64
        npj = n_proj or 60
        P = trajectories.circular_cone(npj, 64, 64, 200.0, 400.0, 1.5)
        return ScanConfig(name, (N, N, N), npj, 64, 64, 1, 0.5, P,
                          extra=dict(fov_radius=22.0, n_ellipsoids=8,
                                     semi=(4.0, 20.0), mu=(0.1, 1.0)))
    if name == "full":
        N = 512
        npj = n_proj or 720
        sod = 3.125 * N
        P = trajectories.circular_cone(npj, 768, 768, sod, 2 * sod, 1.5)
        return ScanConfig(name, (N, N, N), npj, 768, 768, 1, 0.5, P,
                          extra=dict(n_ellipsoids=200, semi=(4.0, 40.0), mu=(0.1, 1.0),
                                     cyl=(0.45 * N, 0.9 * N, 0.1)))
    if name == "helical":
        N = 256
        npj = n_proj or 1200
        sod = 3.125 * N
        sdd = 2 * sod
        n_u, n_v = 512, 256
        p = trajectories.medical_pitch_per_rad(1.0, n_v, 1.5, sod, sdd)
        h_iso = n_v * 1.5 * sod / sdd
        total = (N + h_iso) / p
        rng = np.random.default_rng([seed, 3, 1])
        P = trajectories.helical_cone(npj, n_u, n_v, sod, sdd, 1.5, p, total, n_sub=4)
        P = trajectories.rigid_jitter(P, 0.5, 0.2, rng)
        U = trajectories.smooth_displacement(32, 3.0, np.random.default_rng([seed, 3, 2]))
        tau = trajectories.exposure_time_fractions(npj, 4)
        return ScanConfig(name, (N, N, N), npj, n_u, n_v, 4, 0.5, P, U, tau,
                          extra=dict(n_ellipsoids=32, semi=(16.0, 80.0), mu=(0.1, 1.0),
                                     pitch_per_rad=p, total_angle=total))
    if name in ("diff", "learned"):
        N = 256
        npj = n_proj or (360 if name == "diff" else 180)
        sod = 3.125 * N
        P = trajectories.circular_cone(npj, 384, 384, sod, 2 * sod, 1.5)
        return ScanConfig(name, (N, N, N), npj, 384, 384, 1, 0.5, P,
                          extra=dict(n_ellipsoids=32, semi=(16.0, 80.0), mu=(0.1, 1.0),
                                     I0=1e4, per_width=True))
    raise KeyError(name)


def make_phantom(cfg, seed, supersample=1, dtype=np.float32):
    """Seeded ellipsoid phantom for ``cfg`` (values per voxel, or per volume
    width when the configuration uses noisy transmission data)."""
    rng = np.random.default_rng([seed, 7])
    ex = cfg.extra
    nz, ny, nx = cfg.shape
    fov = ex.get("fov_radius", 0.45 * min(nx, ny))
    ells = phantoms.random_ellipsoids(ex["n_ellipsoids"], cfg.shape, ex["semi"], ex["mu"],
                                      rng, fov_radius=fov)
    vol = phantoms.voxelise_ellipsoids(ells, cfg.shape, supersample=supersample)
    if "cyl" in ex:
        r, h, mu = ex["cyl"]
        vol += phantoms.cylinder_background(cfg.shape, r, h, mu)
    if ex.get("per_width"):
        vol /= float(min(nx, ny))
    return vol.astype(dtype), ells


# Seeds of the learned-correction data sets: disjoint training and test ranges.
TRAIN_SEEDS = range(0, 512)
TEST_SEEDS = range(100000, 100032)


def make_learned_phantom(cfg, seed, device, dtype=None):
    """Training / test phantom of the learned-correction configuration,
    synthesised with torch on ``device``: even seeds give random ellipsoids,
    odd seeds a foam (cylinder of value 0.5 minus spherical voids), both in
    per-volume-width units like ``make_phantom``.  Returns a float64 tensor
    (or ``dtype``) laid out [nz][ny][nx]."""
    import torch
    rng = np.random.default_rng([seed, 7])
    ex = cfg.extra
    nz, ny, nx = cfg.shape
    if seed % 2 == 0:
        fov = ex.get("fov_radius", 0.45 * min(nx, ny))
        ells = phantoms.random_ellipsoids(ex["n_ellipsoids"], cfg.shape, ex["semi"], ex["mu"],
                                          rng, fov_radius=fov)
        vol = phantoms.voxelise_ellipsoids_torch(ells, cfg.shape, device)
    else:
        vol = phantoms.foam_phantom_torch(cfg.shape, rng, device)
    if ex.get("per_width"):
        vol /= float(min(nx, ny))
    return vol if dtype is None else vol.to(dtype)
