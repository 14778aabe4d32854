"""The seeded input generators (no solver arithmetic involved)."""
import numpy as np

import synth


def test_voronoi_is_periodic_nearest_centre():
    rng = np.random.default_rng(0)
    shape = (12, 10, 8)
    g = synth.voronoi_grains(shape, 7, rng)
    assert g.shape == (8, 10, 12) and g.min() >= 0 and g.max() < 7
    rng = np.random.default_rng(0)
    centres = rng.random((7, 3)) * np.array(shape, float)
    z, y, x = 3, 9, 0
    p = np.array([x + 0.5, y + 0.5, z + 0.5])
    d = p - centres
    d -= np.round(d / np.array(shape)) * np.array(shape)
    assert g[z, y, x] == np.argmin((d ** 2).sum(axis=1))


def test_quaternions_unit_positive_w_and_uniform():
    q = synth.random_quaternions(20000, np.random.default_rng(1))
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0)
    assert (q[:, 0] >= 0).all()
    # uniform rotations: <w^2> = 1/4 and rotation angles follow (1 - cos)/pi
    assert abs(np.mean(q[:, 0] ** 2) - 0.25) < 0.01
    ang = 2 * np.arccos(np.clip(q[:, 0], -1, 1))
    assert abs(np.mean(ang) - (np.pi / 2 + 2 / np.pi)) < 0.02


def test_lognormal_density():
    r = synth.lognormal_rho((32, 32, 32), 1e12, 0.3, np.random.default_rng(2))
    l = np.log(r / 1e12)
    assert abs(l.mean()) < 0.01 and abs(l.std() - 0.3) < 0.01


def test_nuclei_match_full_grid_placement_and_sit_on_boundaries():
    g = synth.voronoi_grains((24, 20, 16), 12, np.random.default_rng(3))
    rho = np.full(g.shape, 1e12)
    a = synth.grain_boundary_nuclei(g, rho, 0.05, (3.0, 6.0), 1e10, np.random.default_rng(9))
    rng = np.random.default_rng(9)
    gb = np.zeros(g.shape, bool)
    for ax in range(3):
        for s in (1, -1):
            gb |= g != np.roll(g, s, axis=ax)
    idx = np.flatnonzero(gb)
    cov = np.zeros(g.shape, bool)
    n2, n1, n0 = g.shape
    zz, yy, xx = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    while cov.sum() < 0.05 * g.size:
        c = idx[rng.integers(idx.size)]
        cz, cy, cx = np.unravel_index(c, g.shape)
        r = rng.uniform(3, 6)
        dz = (zz - cz + n2 // 2) % n2 - n2 // 2
        dy = (yy - cy + n1 // 2) % n1 - n1 // 2
        dx = (xx - cx + n0 // 2) % n0 - n0 // 2
        cov |= dx * dx + dy * dy + dz * dz <= r * r
    assert np.array_equal(a == 1e10, cov)
    assert 0.05 <= cov.mean() < 0.05 + 4 * np.pi * 6 ** 3 / 3 / g.size


def test_workloads_are_seeded():
    w = synth.Workload("t", (8, 8, 8), 4, "lognormal", 1, 1e-6, seed=11)
    q1, r1, g1 = synth.make_microstructure(w)
    q2, r2, g2 = synth.make_microstructure(w)
    assert np.array_equal(q1, q2) and np.array_equal(r1, r2) and np.array_equal(g1, g2)
    assert q1.shape == (4, 8, 8, 8)
