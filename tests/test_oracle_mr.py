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


# ---------------------------------------------------------------------------
# Eq. 6 term by term, Eq. 4-5 with GND densities, Eq. 11 with the mobile
# density: values worked out by hand in SI units (J, Pa, m), so that a unit
# slip (MPa taken for Pa: a factor 1e6) or a flipped sign fails.
# ---------------------------------------------------------------------------
KB_HAND = 1.380649e-23


def one_voxel(x):
    return np.full((1, 12), float(x))


def eq6_terms(T):
    """rho_SSD 1e12, rho_F 5e12, rho_P 8e12 m^-2, tau 20 MPa, gdot 1e-3 /s,
    sigma_vm 60 MPa, gdot_vm 2e-3 /s, Table 1 constants, mu 47,337 MPa,
    b 2.56e-10 m, nu 0.34:
      lock forming   c4 sqrt(rho_F) gdot = 8e7 * 2.2360680e6 * 1e-3 = 1.7888544e11
      dipole         d = sqrt3 mu b / (16 pi (1-nu) tau)
                       = 1.7320508 * 47.337e9 * 2.56e-10 / (16 pi 0.66 * 20e6) = 3.1634250e-8 m;
                     rho_M = 2 kT / (c1 c2 c3 mu b^3) sqrt(rho_P rho_F)
                       = 2 kT / (4.5 * 47.337e9 * 1.6777216e-29) * 6.3245553e12
                       (473 K: kT = 6.5304698e-21 J -> 2.3113796e10; 723 K: 3.5330390e10);
                     c6 d rho_M gdot = 3e10 * 3.1634250e-8 * rho_M * 1e-3
                       (473 K: 2.1935628e10; 723 K: 3.3529511e10)
      athermal       -c5 rho_SSD gdot = -1e10
      climb          -c7 exp(-Q_bulk/kT) (sigma_vm/kT) rho_SSD^2 gdot_vm^c8,
                     (2e-3)^0.24 = 0.2250426; 473 K: exp(-53.748) = 4.5448496e-24,
                     60e6/kT = 9.1877e27 m^-3 -> 6.5776625; 723 K: 5.0721437e8."""
    return {473.0: (1.7888543820e11, 2.1935627668e10, -1.0e10, -6.5776624597),
            723.0: (1.7888543820e11, 3.3529511214e10, -1.0e10, -5.0721437196e8)}[T]


@pytest.mark.parametrize("T", [473.0, 723.0])
def test_ssd_rate_terms_by_hand(T):
    full = replace(MR.MaRoters(), T=T)
    args = (one_voxel(1e12), one_voxel(5e12), one_voxel(8e12), one_voxel(20.0), one_voxel(1e-3),
            np.array([60.0]), np.array([2e-3]))
    want = eq6_terms(T)
    only = [dict(c5=0.0, c6=0.0, c7=0.0), dict(c4=0.0, c5=0.0, c7=0.0),
            dict(c4=0.0, c6=0.0, c7=0.0), dict(c4=0.0, c5=0.0, c6=0.0)]
    for term, zero in zip(want, only):
        got = MR.ssd_rates(replace(full, **zero), *args)
        assert np.allclose(got, term, rtol=1e-9, atol=0), (zero, got[0, 0], term)
    got = MR.ssd_rates(full, *args)
    assert np.allclose(got, sum(want), rtol=1e-9, atol=0)
    # the terms take |gdot| and |tau|: a negative slip rate and shear give the same rates
    neg = (args[0], args[1], args[2], -args[3], -args[4], args[5], args[6])
    assert np.allclose(MR.ssd_rates(full, *neg), got, rtol=1e-14, atol=0)


def test_mobile_density_is_a_small_fraction():
    """The paper remarks that the mobile population is a small fraction of the
    immobile one; the reading of rho_M gives, at 473 K with a voxel's density
    split equally over the systems, rho_M / rho_SSD = 2 kT sqrt(4 sqrt2
    (4 + 2 sqrt7)) / (c1 c2 c3 mu b^3) = 0.026495 (worked out by hand); the
    oracle's total density of Eq. 11 carries exactly that excess."""
    from oracle import drx as DX
    law = MR.MaRoters()
    ssd = np.full((1, 12), 1e12 / 12)
    zero = np.zeros((12, 1))
    k = DX.total_density(np.array([1e12]), zero, zero, law, ssd)
    assert abs((k[0] - 1e12) / 1e12 - 0.026495477451) < 1e-10


def test_projections_with_gnd_by_hand():
    """Eq. 4-5 with a screw GND density 3 and an edge GND density 4 on system
    0 (n = (1,1,1)/sqrt3, d = (0,1,-1)/sqrt2, t = n x d = (-2,1,1)/sqrt6) and
    no SSD: rho_F^a = 3 |n^a.d^0| + 4 |n^a.t^0|, rho_P^a the same with the
    sines. |n.d0|: 0 on planes (111), (-111); sqrt(2/3) on (1-11), (11-1).
    |n.t0|: 0 on (111); 2 sqrt2/3 on (-111); sqrt2/3 on (1-11), (11-1)."""
    gs = np.zeros((1, 12)); ge = np.zeros((1, 12))
    gs[0, 0], ge[0, 0] = 3.0, -4.0     # the sign of a GND density does not matter
    F, P = MR.projections(np.zeros((1, 12)), gs, ge)
    r23, r2 = np.sqrt(2.0 / 3.0), np.sqrt(2.0)
    wantF = np.array([0.0] * 3 + [4 * 2 * r2 / 3] * 3 + [3 * r23 + 4 * r2 / 3] * 6)
    wantP = np.array([3.0 + 4.0] * 3 + [3.0 + 4.0 / 3] * 3
                     + [3 * np.sqrt(1.0 / 3.0) + 4 * np.sqrt(7.0) / 3] * 6)
    assert np.allclose(F[0], wantF, rtol=1e-14, atol=1e-14)
    assert np.allclose(P[0], wantP, rtol=1e-14, atol=1e-14)
