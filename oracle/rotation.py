"""Lattice rotation from the plastic spin — TEST INFRASTRUCTURE ONLY.

The microstructure update of Sec. 2.5 names the change of lattice
orientation due to deformation without giving its equation. Reading (the
standard crystal-plasticity kinematics): the lattice spins with
    Omega_e = W - Omega_p,   Omega_p = sum_a gdot_a skew(d_a (x) n_a),
d_a and n_a the unit slip direction and plane normal rotated into the sample
frame, W the local total spin. The local fluctuation of W (the
antisymmetric part of the displacement gradient of the spectral solution) is
not computed: W is the imposed macroscopic spin, zero for the loadings here
(no rigid rotation is applied). Over an increment the orientation becomes
    R <- expm(dt Omega_e) R,
with the converged slip rates of the increment (those that advance the
plastic strain).

Arrays: quaternions (4, V) (w, x, y, z), slip rates (V, 12).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from .crystal import slip_systems
from .tensors import quat_to_rot


def lattice_spin(quat, gdot):
    """Omega_e (V, 3, 3), sample frame, zero imposed spin."""
    n, d = slip_systems()
    R = quat_to_rot(quat)                                   # (V, 3, 3)
    ns = np.einsum("vij,aj->vai", R, n)
    ds = np.einsum("vij,aj->vai", R, d)
    dn = np.einsum("vai,vaj->vaij", ds, ns)
    skew = 0.5 * (dn - np.swapaxes(dn, -1, -2))
    return -np.einsum("va,vaij->vij", np.asarray(gdot, dtype=np.float64), skew)


def rot_to_quat(R):
    """Rotation matrices (V, 3, 3) -> unit quaternions (4, V), w >= 0
    (Shepperd's branch on the largest of w^2, x^2, y^2, z^2)."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty((R.shape[0], 4))
    for v in range(R.shape[0]):
        m = R[v]
        t = np.trace(m)
        cand = np.array([1 + t, 1 + 2 * m[0, 0] - t, 1 + 2 * m[1, 1] - t, 1 + 2 * m[2, 2] - t])
        k = int(np.argmax(cand))
        s = 2.0 * np.sqrt(cand[k])
        if k == 0:
            q = [s / 4, (m[2, 1] - m[1, 2]) / s, (m[0, 2] - m[2, 0]) / s, (m[1, 0] - m[0, 1]) / s]
        elif k == 1:
            q = [(m[2, 1] - m[1, 2]) / s, s / 4, (m[0, 1] + m[1, 0]) / s, (m[0, 2] + m[2, 0]) / s]
        elif k == 2:
            q = [(m[0, 2] - m[2, 0]) / s, (m[0, 1] + m[1, 0]) / s, s / 4, (m[1, 2] + m[2, 1]) / s]
        else:
            q = [(m[1, 0] - m[0, 1]) / s, (m[0, 2] + m[2, 0]) / s, (m[1, 2] + m[2, 1]) / s, s / 4]
        q = np.array(q)
        out[v] = q if q[0] >= 0 else -q
    return out.T


def rotate(quat, gdot, dt):
    """Orientations after an increment: R <- expm(dt Omega_e) R."""
    W = lattice_spin(quat, gdot)
    R = quat_to_rot(quat)
    Rn = np.array([expm(dt * W[v]) @ R[v] for v in range(R.shape[0])])
    return rot_to_quat(Rn)
