"""Pins of the oracle's lattice rotation (plastic spin, zero imposed spin):
the textbook single-slip rotations (in compression the slip-plane normal
turns towards the load axis, in tension the slip direction does), no slip no
rotation, unit quaternions, and the matrix/quaternion round trip."""
import numpy as np

from oracle import rotation as ROT
from oracle.crystal import slip_systems
from oracle.tensors import quat_to_rot


def q_axis_angle(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.array([np.cos(ang / 2), *(np.sin(ang / 2) * a)])


def single_slip(quat, a, sense):
    """Slip rate of system a with the sign a uniaxial load of the given sense
    (-1 compression, +1 tension along z) gives it."""
    n, d = slip_systems()
    R = quat_to_rot(quat[:, None])[0]
    schmid = (R @ d[a])[2] * (R @ n[a])[2]
    g = np.zeros((1, 12))
    g[0, a] = 1e-3 * np.sign(schmid) * sense
    return g


def angle_to_z(v):
    return np.degrees(np.arccos(abs(v[2]) / np.linalg.norm(v)))


def test_single_slip_textbook_rotations():
    rng = np.random.default_rng(5)
    n, d = slip_systems()
    for _ in range(20):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        a = int(rng.integers(12))
        R0 = quat_to_rot(q[:, None])[0]
        if abs((R0 @ d[a])[2] * (R0 @ n[a])[2]) < 0.1:
            continue
        qc = ROT.rotate(q[:, None], single_slip(q, a, -1), 10.0)[:, 0]
        Rc = quat_to_rot(qc[:, None])[0]
        assert angle_to_z(Rc @ n[a]) < angle_to_z(R0 @ n[a])     # normal towards the axis
        qt = ROT.rotate(q[:, None], single_slip(q, a, +1), 10.0)[:, 0]
        Rt = quat_to_rot(qt[:, None])[0]
        assert angle_to_z(Rt @ d[a]) < angle_to_z(R0 @ d[a])     # direction towards the axis


def test_no_slip_no_rotation_and_unit_quaternions():
    rng = np.random.default_rng(6)
    q = rng.normal(size=(4, 7))
    q /= np.linalg.norm(q, axis=0)
    q[:, q[0] < 0] *= -1
    assert np.allclose(ROT.rotate(q, np.zeros((7, 12)), 2.0), q, atol=1e-14)
    qn = ROT.rotate(q, rng.normal(size=(7, 12)) * 1e-3, 2.0)
    assert np.allclose(np.linalg.norm(qn, axis=0), 1.0, atol=1e-14)


def test_quaternion_round_trip_and_small_rotation_angle():
    rng = np.random.default_rng(7)
    q = rng.normal(size=(4, 50))
    q /= np.linalg.norm(q, axis=0)
    q[:, q[0] < 0] *= -1
    assert np.allclose(ROT.rot_to_quat(quat_to_rot(q)), q, atol=1e-13)
    # rotation about z by 90 degrees
    qz = q_axis_angle([0, 0, 1], np.pi / 2)
    assert np.allclose(ROT.rot_to_quat(quat_to_rot(qz[:, None]))[:, 0], qz, atol=1e-15)
    # the spin's magnitude: one system, rate g, turns the lattice by |g| dt / 2
    # about the sense vector n x d (the plastic spin's axial vector)
    g = np.zeros((1, 12))
    g[0, 0] = 2e-3
    q0 = np.array([[1.0], [0.0], [0.0], [0.0]])
    q1 = ROT.rotate(q0, g, 1.0)[:, 0]
    n, d = slip_systems()
    t = np.cross(n[0], d[0])
    ang = 2 * np.arccos(q1[0])
    assert abs(ang - 1e-3) < 1e-12
    axis = q1[1:] / np.linalg.norm(q1[1:])
    assert abs(abs(axis @ t) - 1) < 1e-12


def _random_displacement_modes(shape, rng, nmodes=6):
    """A periodic displacement of a few random Fourier modes (no index at
    N/2) and its exact strain and rotation fields, from the derivative of
    each mode written out (not from the strain)."""
    n0, n1, n2 = shape
    z, y, x = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    u = np.zeros((n2, n1, n0, 3))
    G = np.zeros((n2, n1, n0, 3, 3))       # du_i / dx_j in units of the grid
    for _ in range(nmodes):
        k = np.array([rng.integers(-n0 // 2 + 1, n0 // 2), rng.integers(-n1 // 2 + 1, n1 // 2),
                      rng.integers(-n2 // 2 + 1, n2 // 2)])
        if not k.any():
            continue
        xi = 2 * np.pi * k / np.array([n0, n1, n2])
        a, b = rng.normal(size=3), rng.normal(size=3)
        ph = xi[0] * x + xi[1] * y + xi[2] * z
        u += np.cos(ph)[..., None] * a + np.sin(ph)[..., None] * b
        G += (-np.sin(ph)[..., None, None] * a[:, None] + np.cos(ph)[..., None, None] * b[:, None]) * xi[None, :]
    eps = 0.5 * (G + np.swapaxes(G, -1, -2))
    w = 0.5 * (G - np.swapaxes(G, -1, -2))
    return eps.reshape(-1, 3, 3), w.reshape(-1, 3, 3)


def test_local_rotation_of_a_displacement_field():
    """The rotation recovered from the strain alone equals the antisymmetric
    part of the displacement gradient, computed mode by mode from the
    displacement, on a cubic and a non-cubic grid; a uniform strain carries
    none; the mean local rotation is zero."""
    from oracle.tensors import tensor_to_mandel
    rng = np.random.default_rng(12)
    for shape in ((8, 8, 8), (16, 8, 4)):
        eps, w = _random_displacement_modes(shape, rng)
        got = ROT.local_rotation(tensor_to_mandel(eps), shape)
        assert np.abs(got - w).max() < 1e-12 * np.abs(w).max()
        assert np.abs(got.mean(axis=0)).max() < 1e-14 * np.abs(w).max()
        uni = np.tile(tensor_to_mandel(eps[:1]), (eps.shape[0], 1))
        assert np.abs(ROT.local_rotation(uni, shape)).max() < 1e-15


def test_simple_shear_mode_rotates_by_half_the_shear():
    """u_x = g sin(2 pi y / n1): the local rotation about z is
    w_xy = (1/2) du_x/dy (the textbook split of a simple shear into strain
    and rotation), so its axial component about z is -(1/2) du_x/dy."""
    from oracle.tensors import tensor_to_mandel
    shape = (4, 16, 4)
    n1 = 16
    y = np.arange(n1)
    g = 1e-3
    dudy = g * 2 * np.pi / n1 * np.cos(2 * np.pi * y / n1)
    eps = np.zeros((4, n1, 4, 3, 3))
    eps[..., 0, 1] = eps[..., 1, 0] = 0.5 * dudy[None, :, None]
    w = ROT.local_rotation(tensor_to_mandel(eps.reshape(-1, 3, 3)), shape).reshape(4, n1, 4, 3, 3)
    assert np.allclose(w[..., 0, 1], 0.5 * dudy[None, :, None], rtol=0, atol=1e-17)
    assert np.allclose(w[..., 1, 0], -0.5 * dudy[None, :, None], rtol=0, atol=1e-17)
    assert np.abs(w[..., 2, :]).max() < 1e-18 and np.abs(w[..., :, 2]).max() < 1e-18


def test_rotation_combines_local_and_plastic_spin():
    """With no slip the lattice turns by the local rotation alone (a rotation
    by |w| about its axis); with both, expm of their sum."""
    from scipy.linalg import expm
    q = q_axis_angle([1, 2, 3], 0.4)[:, None]
    dw = np.zeros((1, 3, 3))
    dw[0, 0, 1], dw[0, 1, 0] = -2e-3, 2e-3          # 2e-3 rad about +z
    qn = ROT.rotate(q, np.zeros((1, 12)), 2.0, dw)
    want = q_axis_angle([0, 0, 1], 2e-3)
    from oracle.tensors import quat_to_rot
    Rn = quat_to_rot(qn)[0]
    assert np.allclose(Rn, quat_to_rot(want[:, None])[0] @ quat_to_rot(q)[0], atol=1e-15)
    g = np.random.default_rng(3).normal(size=(1, 12)) * 1e-4
    qb = ROT.rotate(q, g, 2.0, dw)
    Wp = 2.0 * ROT.lattice_spin(q, g)[0]
    assert np.allclose(quat_to_rot(qb)[0], expm(Wp + dw[0]) @ quat_to_rot(q)[0], atol=1e-15)
