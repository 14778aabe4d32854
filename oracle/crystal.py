"""Crystal geometry and the per-voxel material of the oracle (test infrastructure only).

* Slip systems: the 12 FCC {111}<110> systems (Sec. 2.1, Eq. 2 sums over the
  active slip systems; their geometry is the FCC one of Sec. 2.2). Each
  system has unit normal n and unit direction d with n.d = 0; shear is signed,
  so each system is listed once (12, not 24).
* Schmid tensor m = sym(d (x) n), rotated to the sample frame with the voxel
  orientation (Eq. 2).
* Elastic stiffness C(x): cubic constants rotated by the voxel orientation
  (Eq. 1, anisotropic elasticity); compliance S(x) = C(x)^-1.
"""
from __future__ import annotations

import numpy as np

from .tensors import (c4_to_mandel, cubic_c4, quat_to_rot, rotate_c4,
                      tensor_to_mandel)

_N = np.array([[1, 1, 1], [-1, 1, 1], [1, -1, 1], [1, 1, -1]], dtype=np.float64)
_D = {
    0: [[0, 1, -1], [1, 0, -1], [1, -1, 0]],
    1: [[0, 1, -1], [1, 0, 1], [1, 1, 0]],
    2: [[0, 1, 1], [1, 0, -1], [1, 1, 0]],
    3: [[0, 1, 1], [1, 0, 1], [1, -1, 0]],
}


def slip_systems():
    """(normals, directions), each (12, 3), unit vectors in the crystal frame."""
    ns, ds = [], []
    for p in range(4):
        for d in _D[p]:
            ns.append(_N[p] / np.sqrt(3.0))
            ds.append(np.asarray(d, dtype=np.float64) / np.sqrt(2.0))
    return np.array(ns), np.array(ds)


def schmid_sample(R):
    """Mandel Schmid vectors in the sample frame, shape (M, 12, 6)."""
    n, d = slip_systems()
    nr = np.einsum("mij,aj->mai", R, n)
    dr = np.einsum("mij,aj->mai", R, d)
    T = 0.5 * (np.einsum("mai,maj->maij", dr, nr) + np.einsum("mai,maj->maij", nr, dr))
    return tensor_to_mandel(T)


def voxel_material(quat, C11, C12, C44):
    """Per-voxel Mandel stiffness, compliance and Schmid vectors.

    ``quat`` has shape (4, M). Voxels with identical quaternions share one
    evaluation (a grain map repeats orientations); the arithmetic per
    orientation is unchanged.
    Returns (C (M,6,6), S (M,6,6), m (M,12,6)).
    """
    q = np.asarray(quat, dtype=np.float64).reshape(4, -1)
    uq, inv = np.unique(q.T, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    R = quat_to_rot(uq.T)
    Cc = cubic_c4(C11, C12, C44)
    C = c4_to_mandel(rotate_c4(Cc, R))
    S = np.linalg.inv(C)
    m = schmid_sample(R)
    return C[inv], S[inv], m[inv]
