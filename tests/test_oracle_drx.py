"""Pins of the oracle's DRX nucleation (Sec. 2.3, 2.5): the Weibull law of
the nucleation strength, grain-boundary sites worked out by hand, the
propensity and the event rules."""
import math

import numpy as np

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
