"""Pins of the oracle's version of the paper's own constitutive law (Sec. 2.2,
Eq. 3-6): interaction angles worked out by hand, the elastic range below the
passing stress, the viscoplastic steady state of a single crystal against
the closed form of Eq. 3, and the symmetry of the SSD evolution."""
from dataclasses import replace

import numpy as np
import pytest

from oracle import Oracle, Loading
from oracle import ma_roters as MR

IDQ = np.array([1.0, 0.0, 0.0, 0.0])


def test_interaction_angles_by_hand():
    """n0 = (1,1,1)/sqrt3; system 3 has n = (-1,1,1)/sqrt3, d = (0,1,-1)/sqrt2,
    t = n x d = (-2,-1,-1)/sqrt6: |cos| = 4/sqrt18 = 2 sqrt2/3, |sin| = 1/3.
    Coplanar systems: t and d lie in the plane, cos = 0. Each of the three
    other planes contributes |cos| values 2 sqrt2/3, sqrt2/3, sqrt2/3 and
    |sin| values 1/3, sqrt7/3, sqrt7/3, so the row sums are 4 sqrt2 and
    3 + 1 + 2 sqrt7."""
    cnt, snt, cnd, snd = MR.interaction_tables()
    assert abs(cnt[0, 3] - 2 * np.sqrt(2) / 3) < 1e-15
    assert abs(snt[0, 3] - 1 / 3) < 1e-15
    for a in range(12):
        p = a // 3
        assert np.allclose(cnt[a, 3 * p:3 * p + 3], 0, atol=1e-15)
        assert np.allclose(cnd[a, 3 * p:3 * p + 3], 0, atol=1e-15)
    assert np.allclose(cnt.sum(axis=1), 4 * np.sqrt(2), rtol=1e-14)
    assert np.allclose(snt.sum(axis=1), 4 + 2 * np.sqrt(7), rtol=1e-14)


def single_crystal(law, rho_total, dt, rate=1e-3):
    shape = (8, 8, 8)
    V = 512
    quat = np.repeat(IDQ[:, None], V, axis=1)
    o = Oracle(shape, quat, np.full(V, rho_total))
    o.enable_mr(law)
    return o, Loading(Edot=np.array([0, 0, -rate, 0, 0, 0.0]), dt=dt)


def hand_parameters(law, rho_each):
    kT = MR.KB * law.T
    rF, rP = 4 * np.sqrt(2) * rho_each, (4 + 2 * np.sqrt(7)) * rho_each
    tp = law.c1 * law.mu * law.b * np.sqrt(rP)
    tc = law.Qslip / (law.c2 * law.c3 * law.b ** 2) * np.sqrt(rF) * 1e-6
    A = 2 * kT / (law.c1 * law.c3 * law.mu * 1e6 * law.b ** 2) * law.nuD * np.sqrt(rP) * np.exp(-law.Qslip / kT)
    return tp, tc, A


def test_elastic_below_the_passing_stress():
    """A strain of 1e-5 along [001] stays below sqrt6 tau_pass: the response
    is the cubic crystal's Young's modulus E[001] = 66,688.75 MPa."""
    law = MR.MaRoters()
    o, load = single_crystal(law, 2.5e12, dt=1e-2)
    r = o.increment(load, tol=1e-12, max_iter=200)
    assert abs(r["Sigma"][2] / r["E"][2] - 66688.75) < 1e-6 * 66688.75
    assert np.abs(o.epsp).max() == 0.0


def test_single_crystal_steady_state_closed_form():
    """Densities frozen (c4 = c5 = c6 = c7 = 0): at steady state the plastic
    rate carries the applied rate, 8 systems at Schmid factor 1/sqrt6 give
    |sigma33| = sqrt6 (tau_pass + tau_cut asinh(sqrt6 rate / (8 A)))."""
    law = replace(MR.MaRoters(), c4=0.0, c5=0.0, c6=0.0, c7=0.0)
    rho = 2.5e12
    o, load = single_crystal(law, rho, dt=2.0)
    for _ in range(6):
        r = o.increment(load, tol=1e-12, max_iter=500)
    tp, tc, A = hand_parameters(law, rho / 12)
    want = np.sqrt(6) * (tp + tc * np.arcsinh(np.sqrt(6) * 1e-3 / (8 * A)))
    assert abs(-r["Sigma"][2] - want) < 1e-9 * want


def test_ssd_evolution_symmetry_under_001_compression():
    """Under [001] compression of an unrotated crystal the 8 loaded systems
    harden alike and the 4 unloaded ones (Schmid factor 0) alike; only the
    loaded ones store dislocations (lock forming, c4), the unloaded ones lose
    density by climb only."""
    law = MR.MaRoters()
    o, load = single_crystal(law, 2.5e12, dt=2.0)
    for _ in range(2):
        o.increment(load, tol=1e-10, max_iter=500)
    ssd = o.field("rho_ssd")[:, 0]
    from oracle.crystal import slip_systems
    n, d = slip_systems()
    loaded = np.abs(n[:, 2] * d[:, 2]) > 0.1
    assert loaded.sum() == 8
    assert np.ptp(ssd[loaded]) < 1e-9 * ssd[loaded].max()
    assert np.ptp(ssd[~loaded]) < 1e-9 * ssd[~loaded].max()
    assert ssd[loaded].min() > 2.5e12 / 12 > ssd[~loaded].max()
