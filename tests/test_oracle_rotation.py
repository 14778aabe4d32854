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
