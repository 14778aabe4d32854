"""Pins of the oracle's GND update (Sec. 2.2, Eq. 7-8) against values fixed
independently of it: exact differences of linear fields, grain-boundary
stencils, hand-computed sense vectors, rotation invariance, the textbook von
Mises strain and the single-crystal limit."""
import numpy as np

from oracle import Oracle, Loading
from oracle.gnd import grain_difference, gnd_rates, next_leff, sense_vectors, von_mises_strain
from oracle.tensors import quat_to_rot, voigt_to_mandel


def octant_grains(n=16):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return (x >= n // 2) * 1 + (y >= n // 2) * 2 + (z >= n // 2) * 4, x, y, z


def test_linear_field_exact_inside_grains():
    """Octant grains, f = a x + b y + c z: every difference stays inside a
    grain (the periodic wrap crosses a grain boundary), so central and
    one-sided differences are both exact."""
    gr, x, y, z = octant_grains()
    a, b, c = 3.0, -2.0, 0.5
    f = (a * x + b * y + c * z)[None].astype(float)
    assert np.allclose(grain_difference(f, gr, -1), a, atol=1e-12)
    assert np.allclose(grain_difference(f, gr, -2), b, atol=1e-12)
    assert np.allclose(grain_difference(f, gr, -3), c, atol=1e-12)


def test_piecewise_constant_field_has_no_gradient():
    """Constant per grain: central differences across a boundary would see
    the jump; the grain-aware stencil must not."""
    gr, *_ = octant_grains()
    f = (10.0 * gr + 1.0)[None]
    for ax in (-1, -2, -3):
        assert np.abs(grain_difference(f, gr, ax)).max() == 0.0


def test_one_voxel_grain_and_one_sided_values():
    n = 8
    gr = np.zeros((n, n, n), int)
    gr[:, :, 3] = 1                      # a one-voxel-thick grain along x
    gr[:, :, 6:] = 2                     # a two-voxel grain (x = 6, 7)
    f = np.zeros((1, n, n, n))
    f[..., :] = np.arange(n) ** 2        # f = x^2
    d = grain_difference(f, gr, -1)[0, 0, 0]
    assert d[3] == 0.0                   # no in-grain neighbour
    assert d[6] == 49.0 - 36.0           # forward (x = 5 is in grain 0)
    assert d[7] == 49.0 - 36.0           # backward (x = 0 is in grain 0)
    assert d[1] == (4.0 - 0.0) / 2       # central
    assert d[2] == 4.0 - 1.0             # backward (x = 3 is grain 1)
    assert d[4] == 25.0 - 16.0           # forward (x = 3 is grain 1)
    assert d[0] == 1.0 - 0.0             # forward (x = -1 -> 7 is grain 2)


def test_sense_vector_of_first_system_and_rates():
    """System 0: n = (1,1,1)/sqrt3, d = (0,1,-1)/sqrt2, t = n x d =
    (-2,1,1)/sqrt6 (by hand). A linear slip-rate field with gradient g/h per
    metre gives rhodot_s = -(g.t)/(b h), rhodot_et = (g.d)/(b h)."""
    n, d, t = sense_vectors()
    assert np.allclose(t[0], np.array([-2, 1, 1]) / np.sqrt(6), atol=1e-15)
    assert np.allclose(np.abs(np.einsum("ai,ai->a", t, n)), 0, atol=1e-15)
    assert np.allclose(np.abs(np.einsum("ai,ai->a", t, d)), 0, atol=1e-15)
    gr, x, y, z = octant_grains()
    g = np.array([3.0, -2.0, 0.5])
    field = np.tile((g[0] * x + g[1] * y + g[2] * z).reshape(1, -1), (12, 1)) * 1e-6
    V = field.shape[1]
    quat = np.tile(np.array([1.0, 0, 0, 0])[:, None], (1, V))
    b, h = 2.5e-10, 2e-5
    rs, ret = gnd_rates(field, quat, gr, (16, 16, 16), b, h)
    gphys = g * 1e-6 / h
    want_s0 = -(gphys @ np.array([-2, 1, 1]) / np.sqrt(6)) / b
    want_e0 = (gphys @ np.array([0, 1, -1]) / np.sqrt(2)) / b
    assert np.allclose(rs[0], want_s0, rtol=1e-12)
    assert np.allclose(ret[0], want_e0, rtol=1e-12)


def test_rates_rotate_with_the_crystal():
    """Rotating the lattice and the slip-rate gradient together leaves the
    rates unchanged; the screw and edge parts are the projections of the
    gradient on the orthonormal (t, d) pair."""
    gr, x, y, z = octant_grains()
    g = np.array([1.0, 2.0, -0.7])
    ang = 0.7
    ax = np.array([1.0, 2.0, 3.0]) / np.sqrt(14)
    q = np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * ax])
    R = quat_to_rot(q[:, None])[0]
    gr_rot = R @ g
    V = 16 ** 3
    f0 = np.tile((g[0] * x + g[1] * y + g[2] * z).reshape(1, -1), (12, 1))
    f1 = np.tile((gr_rot[0] * x + gr_rot[1] * y + gr_rot[2] * z).reshape(1, -1), (12, 1))
    qI = np.tile(np.array([1.0, 0, 0, 0])[:, None], (1, V))
    qR = np.tile(q[:, None], (1, V))
    a0 = gnd_rates(f0, qI, gr, (16,) * 3, 1.0, 1.0)
    a1 = gnd_rates(f1, qR, gr, (16,) * 3, 1.0, 1.0)
    assert np.allclose(a0[0], a1[0], rtol=1e-12, atol=1e-12)
    assert np.allclose(a0[1], a1[1], rtol=1e-12, atol=1e-12)
    # |proj| <= |grad|, equality for systems whose normal is orthogonal to g
    n, _, _ = sense_vectors()
    tot = a0[0][:, 0] ** 2 + a0[1][:, 0] ** 2
    perp = (g @ g) - (n @ g) ** 2
    assert np.allclose(tot, perp, rtol=1e-12)


def test_von_mises_strain_textbook():
    e = 1e-3
    # incompressible uniaxial: eps_vm = e
    assert abs(von_mises_strain(voigt_to_mandel(np.array([-e / 2, -e / 2, e, 0, 0, 0]))) - e) < 1e-18
    # simple shear (tensor shear e): eps_vm = 2 e / sqrt3
    assert abs(von_mises_strain(voigt_to_mandel(np.array([0, 0, 0, 0, 0, e]))) - 2 * e / np.sqrt(3)) < 1e-18
    # hydrostatic: zero
    assert von_mises_strain(voigt_to_mandel(np.array([e, e, e, 0, 0, 0]))) < 1e-20
    assert next_leff(2.0, voigt_to_mandel(np.array([-e / 2, -e / 2, e, 0, 0, 0])), 200.0) == 2.0 * (1 + e / 200.0)


def test_single_crystal_builds_no_gnd_and_leff_follows_eq8():
    """Uniform orientation and density: uniform slip rates, no gradients;
    l_eff multiplies by (1 + eps_vm/xi) after every increment with eps_vm of
    the mean strain after that increment."""
    shape = (8, 8, 8)
    V = 512
    quat = np.tile(np.array([0.9, 0.1, -0.3, 0.2])[:, None] / np.linalg.norm([0.9, 0.1, -0.3, 0.2]), (1, V))
    o = Oracle(shape, quat, np.full(V, 1e12))
    grains = np.zeros(V, int)
    grains[: V // 2] = 1
    o.enable_gnd(grains, 21.4e-6, 200.0)
    leff = 21.4e-6
    for _ in range(3):
        r = o.increment(Loading(), tol=1e-10, max_iter=500)
        leff *= 1 + von_mises_strain(voigt_to_mandel(r["E"])) / 200.0
        assert np.abs(o.field("rho_gnds")).max() < 1e-6 * 1e12
        assert np.abs(o.field("rho_gndet")).max() < 1e-6 * 1e12
    assert abs(o.gnd["leff"] - leff) < 1e-18
