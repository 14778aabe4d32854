"""Lattice rotation from the local and the plastic spin — TEST INFRASTRUCTURE ONLY.

The microstructure update of Sec. 2.5 names the change of lattice
orientation due to deformation without giving its equation. Reading (the
standard crystal-plasticity kinematics of the full-field elasto-viscoplastic
FFT scheme the paper builds on): over an increment the lattice turns by
    dOmega = dw - dt Omega_p,   Omega_p = sum_a gdot_a skew(d_a (x) n_a),
d_a and n_a the unit slip direction and plane normal rotated into the sample
frame, dw the increment of the local rigid rotation: the antisymmetric part
of the gradient of the periodic displacement fluctuation, whose symmetric
part is the compatible strain the spectral solution returns (the imposed
macroscopic spin is zero for the loadings here). For one Fourier mode of a
compatible field e(xi) = sym(i xi (x) u(xi)), with n = xi / |xi|,
    w(xi) = skew(i xi (x) u(xi)),   w_ij = (e n)_i n_j - n_i (e n)_j,
(the displacement follows from e: |xi| u = -2i e n + i n (n.e.n)), so dw is
the inverse transform of that map applied to the transform of the strain
increment; the mean (xi = 0) carries no local rotation, and Nyquist modes,
where the solver's strain is not a gradient, carry none either. Then
    R <- expm(dOmega) R,
with the converged slip rates of the increment (those that advance the
plastic strain).

Arrays: quaternions (4, V) (w, x, y, z), slip rates (V, 12), local rotation
increments (V, 3, 3), strain increments (V, 6) Mandel.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from .crystal import slip_systems
from .tensors import mandel_to_tensor, quat_to_rot


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


def local_rotation(de, shape):
    """Local rigid-rotation increment (V, 3, 3) of a compatible strain
    increment de (V, 6) Mandel on the periodic grid shape (n0, n1, n2):
    w_hat_ij = (e_hat n)_i n_j - n_i (e_hat n)_j per frequency, n the unit
    wave vector of the frequencies (k0/n0, k1/n1, k2/n2) (index k for k <
    N/2, k - N above), zero at xi = 0 and wherever an index is N/2."""
    n0, n1, n2 = shape
    T = mandel_to_tensor(np.asarray(de, dtype=np.float64)).reshape(n2, n1, n0, 3, 3)
    Th = np.fft.fftn(T, axes=(0, 1, 2))
    def freqs(n):
        k = np.arange(n)
        return np.where(k < n // 2, k, k - n).astype(np.float64) / n, (2 * k == n)
    f0, q0 = freqs(n0)
    f1, q1 = freqs(n1)
    f2, q2 = freqs(n2)
    z = np.zeros((n2, n1, n0))                       # arrays are [z][y][x]
    xi = np.stack([z + f0[None, None, :], z + f1[None, :, None], z + f2[:, None, None]], axis=-1)
    nrm = np.linalg.norm(xi, axis=-1)
    skip = (nrm == 0) | q0[None, None, :] | q1[None, :, None] | q2[:, None, None]
    n = np.where(skip[..., None], 0.0, xi / np.where(nrm == 0, 1.0, nrm)[..., None])
    en = np.einsum("zyxij,zyxj->zyxi", Th, n)
    Wh = np.einsum("zyxi,zyxj->zyxij", en, n) - np.einsum("zyxi,zyxj->zyxij", n, en)
    W = np.fft.ifftn(Wh, axes=(0, 1, 2)).real
    return W.reshape(-1, 3, 3)


def rotate(quat, gdot, dt, dw=None):
    """Orientations after an increment: R <- expm(dw - dt Omega_p) R, dw the
    local rotation increment (V, 3, 3) or None (plastic spin alone)."""
    W = dt * lattice_spin(quat, gdot)
    if dw is not None:
        W = W + dw
    R = quat_to_rot(quat)
    Rn = np.array([expm(W[v]) @ R[v] for v in range(R.shape[0])])
    return rot_to_quat(Rn)
