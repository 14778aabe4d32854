"""Pins of the oracle's DRX nucleation (Sec. 2.3, 2.5): the Weibull law of
the nucleation strength, grain-boundary sites worked out by hand, the
propensity and the event rules."""
import math

import numpy as np
import pytest

from oracle import Oracle, Loading
from oracle import drx as DX


def test_weibull_inverse_and_moments():
    """P(kappa < k) = 1 - exp(-(k/kc)^q) at the drawn values reproduces u;
    median kc (ln 2)^(1/q); the sample mean approaches kc Gamma(1 + 1/q)."""
    kc, q = 300e12, 4.4
    u = np.random.default_rng(5).random(200000)
    kap = DX.weibull_strength(u, kc, q)
    assert np.allclose(1.0 - np.exp(-(kap / kc) ** q), u, rtol=0, atol=1e-12)
    assert abs(DX.weibull_strength(0.5, kc, q) - kc * math.log(2) ** (1 / q)) < 1e-3
    assert abs(kap.mean() / (kc * math.gamma(1 + 1 / q)) - 1) < 5e-3


def test_grain_boundary_sites_by_hand():
    """8^3 grid, grain 1 = the slab x in {2, 3}: sites are x = 1, 2, 3, 4 (the
    slab and its neighbours); a slab spanning the periodic box along x has
    no boundary."""
    n = 8
    g = np.zeros((n, n, n), int)
    g[:, :, 2:4] = 1
    m = DX.gb_sites(g.reshape(-1), (n, n, n)).reshape(n, n, n)
    assert set(np.flatnonzero(m[0, 0])) == {1, 2, 3, 4}
    assert np.array_equal(m, np.broadcast_to(m[0, 0], m.shape))
    assert not DX.gb_sites(np.zeros(n ** 3, int), (n, n, n)).any()


def test_total_density_power_law():
    rho = np.array([1.0, 2.0])
    gs = np.zeros((12, 2))
    ge = np.zeros((12, 2))
    gs[0] = [3.0, 0.0]
    ge[0] = [4.0, 0.0]
    ge[5] = [0.0, -2.0]
    assert np.allclose(DX.total_density(rho, gs, ge), [1.0 + 5.0, 2.0 + 2.0])


def test_nucleation_events():
    """Uniform single crystal split into two grains: after plastic
    increments the sites whose propensity exceeds their strength nucleate,
    interior voxels never do, GND densities of the nuclei scale by s_soften,
    nuclei get their own grain id and a strength drawn with s_nucl k_c."""
    shape = (8, 8, 8)
    V = 512
    quat = np.tile(np.array([1.0, 0, 0, 0])[:, None], (1, V))
    o = Oracle(shape, quat, np.full(V, 1e12))
    grains = np.zeros(V, int)
    grains[np.arange(V) % 8 >= 4] = 1          # x >= 4: grain 1
    o.enable_gnd(grains, 21.4e-6, 200.0)
    drx = DX.DRX(kc=1.5e12, q=4.4)
    u0 = np.random.default_rng(7).random(V)
    o.enable_drx(drx, u0)
    o.increment(Loading(), tol=1e-10, max_iter=500)
    G = o.gnd
    rs0, re0, kap0 = G["rs"].copy(), G["ret"].copy(), o.kappa.copy()
    k = DX.total_density(o.rho, G["rs"], G["ret"])
    sites = DX.gb_sites(grains, shape)
    u1 = np.random.default_rng(8).random(V)
    n = o.drx_nucleate(u1)
    hit = sites & (k > kap0)
    assert n == hit.sum() and 0 < n < sites.sum()
    assert not (~sites & (k > kap0) & (o.field("grain") != grains)).any()
    assert np.array_equal(o.field("grain")[hit], -(np.flatnonzero(hit) + 1.0))
    assert np.allclose(G["rs"][:, hit], 0.9 * rs0[:, hit]) and np.allclose(G["ret"][:, ~hit], re0[:, ~hit])
    assert np.allclose(o.kappa[hit], 0.05 * 1.5e12 * (-np.log1p(-u1[hit])) ** (1 / 4.4))
    assert np.array_equal(o.kappa[~hit], kap0[~hit])


def test_total_density_with_mobile_density_by_hand():
    """Eq. 11 with the paper's law: one voxel, density 1e12 split equally over
    the 12 systems, no GND: rho_F = 4 sqrt2 rho_a, rho_P = (4 + 2 sqrt7) rho_a
    (the row sums of the interaction tables), rho_M^a = 0.026495477 rho_a at
    473 K (see test_oracle_mr), so k = 12 (rho_a + rho_M^a) = 1.0264955e12.
    A GND density adds its magnitude sqrt(screw^2 + edge^2) and raises the
    mobile densities through the projections."""
    from oracle import ma_roters as MR
    law = MR.MaRoters()
    ssd = np.full((1, 12), 1e12 / 12)
    zero = np.zeros((12, 1))
    k = DX.total_density(np.array([1e12]), zero, zero, law, ssd)
    assert abs(k[0] - 1.0264954774514e12) < 1e-9 * 1e12
    gs, ge = zero.copy(), zero.copy()
    gs[0], ge[0] = 3e11, 4e11
    k2 = DX.total_density(np.array([1e12]), gs, ge, law, ssd)
    assert k2[0] > k[0] + 5e11


@pytest.mark.parametrize("factor, grows", [(1.6, True), (0.6, False)])
def test_growth_stored_energy_against_capillarity(factor, grows):
    """drx_grow converts the total density to the stored energy of Eq. 14,
    rho zeta mu b^2 (J/m^3), in the phase field's energy unit. In SI a
    recrystallised sphere of radius R in a deformed matrix grows when that
    energy exceeds the capillary pressure 2 omega / R and shrinks below it.
    Coarse sphere of radius 6 voxels (12 PF cells of dx = 1 um), omega =
    0.625 J/m^2, zeta = 0.25: the critical density is 2 omega / (12 dx zeta mu
    b^2) = 1.0417e5 / 7.7558e-10 = 1.3431e14 m^-2; at 1.6x it grows, at 0.6x
    it shrinks."""
    n = 24
    shape = (n, n, n)
    V = n ** 3
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r2 = (x + 0.5 - n / 2) ** 2 + (y + 0.5 - n / 2) ** 2 + (z + 0.5 - n / 2) ** 2
    inside = (r2 <= 36.0).reshape(-1)
    rho_c = 2 * 0.625 / (12 * 1e-6) / (0.25 * 47337e6 * 2.56e-10 ** 2)
    assert abs(rho_c / 1.34306e14 - 1) < 1e-4
    quat = np.tile(np.array([1.0, 0, 0, 0])[:, None], (1, V))
    o = Oracle(shape, quat, np.full(V, factor * rho_c))
    o.enable_gnd(np.where(inside, -1, 0), 21.4e-6, 200.0)
    o.enable_drx(DX.DRX(), np.full(V, 0.5))
    before = o.field("grain").copy()
    changed, rex = o.drx_grow(400, zeta=0.25, omega_gb=0.625, dx=1e-6, K=2, threshold=1e-5)
    after = o.field("grain")
    gained = int(((before == 0) & (after == -1)).sum())
    lost = int(((before == -1) & (after == 0)).sum())
    if grows:
        assert gained > 50 and lost == 0, (gained, lost)
    else:
        assert lost > 50 and gained == 0, (gained, lost)


def _nucleated(law, k12=None):
    from oracle import Flow
    from oracle import ma_roters as MR
    import synth
    shape = (8, 8, 8)
    V = 512
    g = [np.random.default_rng(s) for s in np.random.SeedSequence(3).spawn(4)]
    grains = synth.voronoi_grains(shape, 4, g[0])
    q = synth.random_quaternions(4, g[1])
    quat = np.moveaxis(q[grains], -1, 0).reshape(4, -1).copy()
    o = Oracle(shape, quat, np.full(V, 2.5e12), flow=Flow(k1=k12[0], k2=k12[1]) if k12 else None)
    o.enable_gnd(grains.reshape(-1), 21.4e-6, 200.0)
    if law == 1:
        o.enable_mr(MR.MaRoters())
    o.enable_drx(DX.DRX(kc=3.2e12 if law == 1 else 2.4e12), np.random.default_rng(5).random(V))
    for _ in range(2):
        before = o.mechanical_state()
        r = o.increment(Loading(), tol=1e-10, max_iter=3000)
    n = o.drx_nucleate(np.random.default_rng(6).random(V))
    assert n > 20
    return o, before, r


def test_redistribution_power_law_frozen_density_is_identity():
    """With the power law at a density that does not evolve, nothing the
    repeated solve depends on changed: the committed state comes back
    exactly (same iteration count)."""
    o, before, r = _nucleated(0, (0.0, 0.0))
    s0, e0, p0 = o.sigma.copy(), o.e.copy(), o.epsp.copy()
    rr = o.redistribute(before, Loading(), tol=1e-10, max_iter=3000)
    assert rr["iters"] == r["iters"]
    assert np.array_equal(o.sigma, s0) and np.array_equal(o.e, e0) and np.array_equal(o.epsp, p0)


def test_redistribution_paper_law_changes_only_the_mechanics():
    """Paper's law with GND densities: after nucleation the repeated solve
    moves the stress (the softened nuclei and the increment's hardening
    enter the slip resistances), leaves densities, grains and time alone,
    keeps the mean strain prescribed and <e> = E, and repeating it from the
    same start state gives the same result."""
    o, before, r = _nucleated(1)
    s0 = o.sigma.copy()
    dens = (o.ssd.copy(), o.gnd["rs"].copy(), o.gnd["grains"].copy(), o.t)
    rr = o.redistribute(before, Loading(), tol=1e-10, max_iter=3000)
    assert rr["converged"] and np.abs(o.sigma - s0).max() > 1.0
    assert np.array_equal(o.ssd, dens[0]) and np.array_equal(o.gnd["rs"], dens[1])
    assert np.array_equal(o.gnd["grains"], dens[2]) and o.t == dens[3]
    assert abs(rr["E"][2] - r["E"][2]) < 1e-15
    assert np.abs(o.e.mean(axis=0) - o.E).max() < 1e-12
    s1, p1 = o.sigma.copy(), o.epsp.copy()
    o.redistribute(before, Loading(), tol=1e-10, max_iter=3000)
    assert np.array_equal(o.sigma, s1) and np.array_equal(o.epsp, p1)
