"""DRX nucleation (Sec. 2.3 and the microstructure update of Sec. 2.5) —
TEST INFRASTRUCTURE ONLY.

* Nucleation strength: kappa(x) follows the Weibull law of Eq. 9-10,
  P(kappa < k) = 1 - exp(-(k/k_c)^q); drawn by inverting that distribution
  at caller-supplied uniform numbers u in (0, 1): kappa = k_c (-ln(1-u))^(1/q).
* Propensity: k(x) = rho_tot(x) (Eq. 11), the sum over systems of mobile, SSD
  and GND densities. Readings: the GND density of a system is
  sqrt(rho_GNDs^2 + rho_GNDet^2) (the conservation law stated with Eq. 7,
  rho_GNDen = 0); with the power law, which has one density per voxel and no
  mobile density, k = rho + sum_a rho_GND^a; with the paper's law the mobile
  density is the reading of oracle.ma_roters.
* Sites: grain-boundary grid points (reading: voxels with a face neighbour
  of another grain, periodic).
* Event: a site nucleates when k > kappa. The voxel becomes a new grain
  (reading: a single-voxel grain with its own id, -(voxel index + 1)); its
  GND densities become s_soften times their value (Eq. 16), its SSD
  densities and orientation stay (Sec. 2.5); its kappa is redrawn with
  k_c' = s_nucl k_c from a fresh uniform number. All sites are tested on the
  state after the increment, then updated together.
* Stress redistribution (Sec. 2.5): after the update the equilibrium stress is
  computed again before further loading, with the pre-DRX strain rate
  prescribed (Oracle.redistribute repeats the last increment's solve from its
  start state with the updated slip resistances).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import ma_roters as MR


@dataclass(frozen=True)
class DRX:
    kc: float = 300e12        # m^-2 (Table 2)
    q: float = 4.4            # (Table 2)
    s_nucl: float = 0.05      # (Table 2)
    s_soften: float = 0.9     # (Table 2)


def weibull_strength(u, kc, q):
    """Inverse of P(kappa < k) = 1 - exp(-(k/kc)^q) at u."""
    return kc * (-np.log1p(-np.asarray(u, dtype=np.float64))) ** (1.0 / q)


def gb_sites(grains, shape):
    """Voxels with a face neighbour in another grain (periodic), (V,) bool."""
    n0, n1, n2 = shape
    g = np.asarray(grains).reshape(n2, n1, n0)
    m = np.zeros(g.shape, dtype=bool)
    for ax in range(3):
        for s in (1, -1):
            m |= np.roll(g, s, axis=ax) != g
    return m.reshape(-1)


def total_density(rho, rho_gs, rho_get, law=None, rho_ssd=None):
    """k(x) = rho_tot (Eq. 11). rho: (V,) voxel density; rho_gs, rho_get:
    (12, V) GND densities or None; law: MaRoters with rho_ssd (V, 12) for the
    paper's law (adds the mobile densities)."""
    gnd = 0.0 if rho_gs is None else np.sqrt(rho_gs ** 2 + rho_get ** 2).sum(axis=0)
    if law is None:
        return rho + gnd
    F, P = MR.projections(rho_ssd, None if rho_gs is None else rho_gs.T,
                          None if rho_get is None else rho_get.T)
    kT = MR.KB * law.T
    rho_m = 2.0 * kT / (law.c1 * law.c2 * law.c3 * law.mu * 1e6 * law.b ** 3) * np.sqrt(P * F)
    return rho_m.sum(axis=1) + rho_ssd.sum(axis=1) + gnd


def nucleate(kappa, k, sites, u_new, drx: DRX):
    """(mask of new nuclei, redrawn kappa)."""
    hit = sites & (k > kappa)
    kap = kappa.copy()
    kap[hit] = weibull_strength(u_new[hit], drx.s_nucl * drx.kc, drx.q)
    return hit, kap
