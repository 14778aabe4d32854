"""Seeded synthetic inputs for the FFT-EVP solve.

This module only *draws* inputs: a periodic Voronoi grain map, uniformly
random lattice orientations, and dislocation-density fields. It holds none of
the solver's arithmetic, so both the CPU oracle and the GPU path can take
their inputs from here without sharing any of the method.

The paper runs its solve on a 64^3 periodic voxel grid of a 191-grain copper
RVE built with DREAM3D (Sec. 3, Table 1). That RVE is not available; the
synthetic periodic Voronoi polycrystals below stand in for it.

Conventions
-----------
* Arrays are laid out ``[z][y][x]`` (x fastest), shape ``(n2, n1, n0)``.
* Quaternions are ``(w, x, y, z)`` unit quaternions with ``w >= 0``, stored
  component-major: ``quat[4][n2][n1][n0]``; they rotate crystal -> sample
  (active).
* Dislocation density is in m^-2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree

__all__ = [
    "Workload", "WORKLOADS", "workload", "voronoi_grains", "random_quaternions",
    "lognormal_rho", "grain_boundary_nuclei", "make_microstructure",
    "random_voxel_states", "single_voxel_nuclei",
]


@dataclass(frozen=True)
class Workload:
    """One synthetic loading case: grid, grains, density field and path."""
    name: str
    shape: tuple            # (n0, n1, n2) = (nx, ny, nz)
    n_grains: int
    rho: str                # "uniform" | "lognormal" | "lognormal+nuclei"
    increments: int
    tol: float
    seed: int
    rho_median: float = 1.0e12      # m^-2
    sigma_log: float = 0.3
    nuclei_fraction: float = 0.05
    nuclei_radius: tuple = (3.0, 6.0)
    nuclei_rho: float = 1.0e10
    strain_rate: float = 1.0e-3     # |d eps33/dt|, 1/s (uniaxial compression)
    d_eps: float = 2.0e-3           # strain per increment
    extra: dict = field(default_factory=dict)

    @property
    def dt(self) -> float:
        return self.d_eps / self.strain_rate

    @property
    def voxels(self) -> int:
        return int(np.prod(self.shape))


# The five synthetic polycrystal workloads. Seeds are fixed per workload.
WORKLOADS = {
    "cu16": Workload("cu16", (16, 16, 16), 8, "uniform", 5, 1e-13, seed=1),
    "cu64": Workload("cu64", (64, 64, 64), 100, "lognormal", 50, 1e-6, seed=2),
    "cu128": Workload("cu128", (128, 128, 128), 500, "lognormal", 100, 1e-6, seed=3),
    "cu128adj": Workload("cu128adj", (128, 128, 128), 300, "lognormal", 40, 1e-6, seed=4),
    "cu256": Workload("cu256", (256, 256, 256), 2000, "lognormal+nuclei", 200, 1e-6,
                      seed=5),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def _streams(seed: int):
    """Four independent generators: centres, orientations, density, nuclei."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


def voronoi_grains(shape, n_grains: int, rng: np.random.Generator) -> np.ndarray:
    """Periodic Voronoi grain map, int32 ``[n2][n1][n0]``.

    Centres are uniform in the periodic box (voxel units); a voxel belongs to
    the centre nearest (minimum-image distance) to its centre point
    ``(i + 1/2)``. Exact ties have probability zero for continuous centres.
    """
    n0, n1, n2 = shape
    box = np.array([n0, n1, n2], dtype=np.float64)
    centres = rng.random((n_grains, 3)) * box
    tree = cKDTree(centres, boxsize=box)
    out = np.empty((n2, n1, n0), dtype=np.int32)
    xs = np.arange(n0) + 0.5
    ys = np.arange(n1) + 0.5
    X, Y = np.meshgrid(xs, ys, indexing="xy")           # (n1, n0)
    for z in range(n2):
        pts = np.stack([X.ravel(), Y.ravel(), np.full(X.size, z + 0.5)], axis=1)
        _, idx = tree.query(pts, k=1)
        out[z] = idx.reshape(n1, n0)
    return out


def random_quaternions(n: int, rng: np.random.Generator) -> np.ndarray:
    """``n`` uniformly distributed rotations (Shoemake 1992), shape (n, 4).

    Returned as (w, x, y, z) with w >= 0.
    """
    u1, u2, u3 = rng.random((3, n))
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    q = np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                  b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], axis=1)
    # (x, y, z, w) ordering of the published recipe -> (w, x, y, z)
    q = q[:, [3, 0, 1, 2]]
    q[q[:, 0] < 0] *= -1.0
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def lognormal_rho(shape, median: float, sigma_log: float, rng) -> np.ndarray:
    """i.i.d. per-voxel log-normal density: ``median * exp(sigma_log * Z)``."""
    n0, n1, n2 = shape
    return median * np.exp(sigma_log * rng.standard_normal((n2, n1, n0)))


def grain_boundary_nuclei(grains: np.ndarray, rho: np.ndarray, fraction: float,
                          radius: tuple, rho_nuc: float, rng) -> np.ndarray:
    """Low-density spherical nuclei centred on grain-boundary voxels.

    A grain-boundary voxel has a periodic face neighbour in another grain.
    Nuclei (centre uniform over boundary voxels, radius uniform in
    ``radius``) are added until at least ``fraction`` of all voxels are
    covered; covered voxels get ``rho_nuc``.
    """
    n2, n1, n0 = grains.shape
    gb = np.zeros(grains.shape, dtype=bool)
    for ax in range(3):
        for s in (1, -1):
            gb |= grains != np.roll(grains, s, axis=ax)
    gb_idx = np.flatnonzero(gb)
    out = rho.copy()
    covered = np.zeros(grains.shape, dtype=bool)
    target = fraction * grains.size
    count = 0
    while count < target and gb_idx.size:
        c = gb_idx[rng.integers(gb_idx.size)]
        cz, cy, cx = np.unravel_index(c, grains.shape)
        r = rng.uniform(*radius)
        # voxels within periodic distance r of the centre, found in the
        # centre's bounding box (wrapped indices)
        k = int(np.ceil(r))
        off = np.arange(-k, k + 1)
        dz, dy, dx = np.meshgrid(off, off, off, indexing="ij")
        inside = dx * dx + dy * dy + dz * dz <= r * r
        zi = (cz + dz[inside]) % n2
        yi = (cy + dy[inside]) % n1
        xi = (cx + dx[inside]) % n0
        new = ~covered[zi, yi, xi]
        covered[zi, yi, xi] = True
        count += int(new.sum())
    out[covered] = rho_nuc
    return out


def single_voxel_nuclei(grains: np.ndarray, fraction: float, rng) -> np.ndarray:
    """Grain map with DRX-like nuclei: a random ``fraction`` of the
    grain-boundary voxels (periodic face neighbour in another grain) become
    one-voxel grains with id ``-(flat index + 1)``."""
    gb = np.zeros(grains.shape, dtype=bool)
    for ax in range(3):
        for s in (1, -1):
            gb |= grains != np.roll(grains, s, axis=ax)
    idx = np.flatnonzero(gb)
    pick = idx[rng.random(idx.size) < fraction]
    out = grains.copy().reshape(-1)
    out[pick] = -(pick + 1)
    return out.reshape(grains.shape)


def make_microstructure(w: Workload):
    """(quat[4][n2][n1][n0], rho[n2][n1][n0], grains[n2][n1][n0]) for ``w``."""
    g_c, g_q, g_r, g_n = _streams(w.seed)
    grains = voronoi_grains(w.shape, w.n_grains, g_c)
    qg = random_quaternions(w.n_grains, g_q)
    quat = np.ascontiguousarray(np.moveaxis(qg[grains], -1, 0))
    if w.rho == "uniform":
        rho = np.full(grains.shape, w.rho_median)
    else:
        rho = lognormal_rho(w.shape, w.rho_median, w.sigma_log, g_r)
        if w.rho == "lognormal+nuclei":
            rho = grain_boundary_nuclei(grains, rho, w.nuclei_fraction,
                                        w.nuclei_radius, w.nuclei_rho, g_n)
    return quat, np.ascontiguousarray(rho), grains


def random_voxel_states(n: int, seed: int, stress_scale: float = 60.0,
                        strain_scale: float = 2.0e-3):
    """Independent random per-voxel inputs for local-solve checks.

    Returns dict with quat (4, n), rho (n,), lam (6, n), e (6, n), epsp (6, n)
    as plain tensor components [11, 22, 33, 23, 13, 12] (MPa / strain).
    """
    rng = np.random.default_rng(seed)
    quat = random_quaternions(n, rng).T.copy()
    rho = 1.0e12 * np.exp(0.5 * rng.standard_normal(n))
    lam = stress_scale * rng.standard_normal((6, n))
    e = strain_scale * rng.standard_normal((6, n))
    epsp = 0.2 * strain_scale * rng.standard_normal((6, n))
    epsp[:3] -= epsp[:3].mean(axis=0)
    return {"quat": quat, "rho": rho, "lam": lam, "e": e, "epsp": epsp}
