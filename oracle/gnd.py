"""Geometrically necessary dislocation densities — TEST INFRASTRUCTURE ONLY.

Sec. 2.2, Eq. 7-8, written out plainly:

* per slip system a, the screw and edge-type GND rates follow from the
  gradient of the slip rate field,
      rhodot_GNDs^a  = -(1/b) grad(gdot^a) . t^a
      rhodot_GNDet^a =  (1/b) grad(gdot^a) . d^a
      rhodot_GNDen^a =  0,
  with d^a the slip direction, n^a the plane normal and t^a = n^a x d^a the
  sense vector (reading: the paper names t "sense vector" without giving its
  orientation), all rotated into the sample frame by the voxel orientation;
* the gradient is a finite difference on the voxel grid: central where both
  neighbours along an axis belong to the voxel's grain, one-sided towards the
  neighbour that does where only one does (the passage after Eq. 7), and zero
  where neither does (reading: a one-voxel-thick grain along that axis has no
  in-grain difference); the grid is periodic;
* the grid spacing in the difference is the effective length l_eff, which
  after each increment becomes l_eff (1 + eps_vm / xi) (Eq. 8), eps_vm being
  the von Mises equivalent of the current mean strain E (reading: "current
  average von Mises equivalent strain"); the increment's rates use l_eff from
  its start;
* the densities integrate explicitly over the increment:
  rho <- rho + dt * rhodot, from the slip rates of the converged increment
  (those that also advance the plastic strain).

Arrays: slip-system-major ``(12, V)``, voxels ``[z][y][x]`` (x fastest).
"""
from __future__ import annotations

import numpy as np

from .crystal import slip_systems
from .tensors import quat_to_rot


def sense_vectors():
    """(n, d, t) in the crystal frame, each (12, 3); t = n x d."""
    n, d = slip_systems()
    return n, d, np.cross(n, d)


def grain_difference(f, grains, axis):
    """Finite difference of ``f`` (..., n2, n1, n0) along ``axis`` (grid units).

    Central where both neighbours are in the voxel's grain, forward or
    backward where only one is, zero where neither is. Periodic.
    """
    assert axis < 0, "axis counted from the end (x = -1)"
    fp = np.roll(f, -1, axis=axis)          # f(x + e)
    fm = np.roll(f, 1, axis=axis)           # f(x - e)
    same_p = np.roll(grains, -1, axis=axis) == grains
    same_m = np.roll(grains, 1, axis=axis) == grains
    central = 0.5 * (fp - fm)
    fwd = fp - f
    bwd = f - fm
    return np.where(same_p & same_m, central,
                    np.where(same_p, fwd, np.where(same_m, bwd, 0.0)))


def gnd_rates(gdot, quat, grains, shape, b, h):
    """(rhodot_s, rhodot_et), each (12, V), from slip rates ``gdot`` (12, V).

    ``grains`` (V,) integer grain ids, ``h`` the grid spacing (m), ``b`` the
    Burgers vector length (m).
    """
    n0, n1, n2 = shape
    g = np.asarray(gdot, dtype=np.float64).reshape(12, n2, n1, n0)
    gr = np.asarray(grains).reshape(n2, n1, n0)
    # gradient components along sample x, y, z (array axes -1, -2, -3)
    grad = np.stack([grain_difference(g, gr, -1), grain_difference(g, gr, -2),
                     grain_difference(g, gr, -3)], axis=-1).reshape(12, -1, 3) / h
    _, d, t = sense_vectors()
    R = quat_to_rot(quat)                                  # (V, 3, 3)
    d_s = np.einsum("vij,aj->avi", R, d)                    # (12, V, 3)
    t_s = np.einsum("vij,aj->avi", R, t)
    rs = -np.sum(grad * t_s, axis=-1) / b
    ret = np.sum(grad * d_s, axis=-1) / b
    return rs, ret


def von_mises_strain(E_mandel):
    """sqrt(2/3 E':E') of a Mandel strain vector."""
    E = np.asarray(E_mandel, dtype=np.float64)
    dev = E.copy()
    dev[:3] -= E[:3].mean()
    return float(np.sqrt(2.0 / 3.0 * dev @ dev))


def next_leff(leff, E_mandel, xi):
    """Eq. 8: l_eff (1 + eps_vm / xi)."""
    return leff * (1.0 + von_mises_strain(E_mandel) / xi)
