"""Tensor bookkeeping for the oracle (test infrastructure only).

Symmetric second-order tensors are 6-vectors in Mandel form
``[t11, t22, t33, sqrt2*t23, sqrt2*t13, sqrt2*t12]`` so that the double
contraction ``a:b`` is the dot product and fourth-order tensors with minor
symmetries are 6x6 matrices. Inputs and outputs at the oracle's public
functions are plain tensor components ``[11, 22, 33, 23, 13, 12]``.

Everything here is written from the definitions: the 4th-order cubic
stiffness of the crystal (Sec. 2.1, Eq. 1: anisotropic elasticity), its
rotation into the sample frame ``C_ijkl = R_ia R_jb R_kc R_ld C_abcd``, and
the conversion to Mandel matrices. No shortcut of the GPU path is reused.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)
# Mandel slot -> (i, j) index pair
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
WEIGHT = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


def voigt_to_mandel(t):
    """Plain components [11,22,33,23,13,12] (leading axis) -> Mandel."""
    t = np.asarray(t, dtype=np.float64)
    return t * WEIGHT.reshape((6,) + (1,) * (t.ndim - 1))


def mandel_to_voigt(m):
    m = np.asarray(m)
    return m / WEIGHT.reshape((6,) + (1,) * (m.ndim - 1))


def tensor_to_mandel(T):
    """(..., 3, 3) symmetric -> (..., 6) Mandel."""
    return np.stack([T[..., i, j] * (1.0 if i == j else SQ2) for i, j in PAIRS], axis=-1)


def mandel_to_tensor(m):
    """(..., 6) Mandel -> (..., 3, 3)."""
    m = np.asarray(m)
    T = np.zeros(m.shape[:-1] + (3, 3), dtype=m.dtype)
    for k, (i, j) in enumerate(PAIRS):
        v = m[..., k] if i == j else m[..., k] / SQ2
        T[..., i, j] = v
        T[..., j, i] = v
    return T


def c4_to_mandel(C):
    """(..., 3,3,3,3) with minor symmetries -> (..., 6, 6) Mandel matrix."""
    out = np.empty(C.shape[:-4] + (6, 6), dtype=C.dtype)
    for a, (i, j) in enumerate(PAIRS):
        for b, (k, l) in enumerate(PAIRS):
            out[..., a, b] = C[..., i, j, k, l] * WEIGHT[a] * WEIGHT[b]
    return out


def cubic_c4(C11, C12, C44):
    """Cubic stiffness in the crystal frame as a 3x3x3x3 array (MPa)."""
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            C[i, i, j, j] = C12
        C[i, i, i, i] = C11
    for i in range(3):
        for j in range(3):
            if i != j:
                C[i, j, i, j] = C44
                C[i, j, j, i] = C44
    return C


def isotropic_c4(lam, mu):
    d = np.eye(3)
    return (lam * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))


def quat_to_rot(q):
    """Unit quaternion (w, x, y, z) (leading axis 4) -> rotation matrices.

    Active rotation, crystal -> sample: ``v_sample = R v_crystal``.
    Returns shape (..., 3, 3).
    """
    w, x, y, z = (np.asarray(q[k], dtype=np.float64) for k in range(4))
    R = np.empty(w.shape + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def rotate_c4(C, R):
    """Sample-frame stiffness ``R_ia R_jb R_kc R_ld C_abcd`` for each R."""
    return np.einsum("...ia,...jb,...kc,...ld,abcd->...ijkl", R, R, R, R, C,
                     optimize=True)
