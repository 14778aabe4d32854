"""The paper's dislocation-based crystal plasticity law — TEST INFRASTRUCTURE ONLY.

Sec. 2.2, Eq. 3-6 (the flow rule of Ma and Roters for FCC metals and its
SSD evolution), written out plainly in SI units with stresses passed in MPa:

* forest and parallel densities of system a (Eq. 4-5),
      rho_F^a = sum_b rho_SSD^b |cos(n^a, t^b)| + |rho_GNDs^b cos(n^a, d^b)|
                + |rho_GNDet^b cos(n^a, t^b)|   (+ rho_GNDen term, zero here)
      rho_P^a = the same with |sin|;
* passing stress tau_pass = c1 mu b sqrt(rho_P), cutting stress
  tau_cut = Q_slip / (c2 c3 b^2) sqrt(rho_F), prefactor
  gdot_0 = 2 kB T / (c1 c3 mu b^2) nu_D sqrt(rho_P) (Sec. 2.2);
* flow rule (Eq. 3): gdot = 0 for |tau| <= tau_pass, otherwise
      gdot = gdot_0 exp(-Q_slip / kB T) sinh((|tau| - tau_pass) / tau_cut) sign(tau);
* SSD evolution (Eq. 6) with |gdot| (reading: densities are stored, not
  signed):
      rhodot_SSD = c4 sqrt(rho_F) |gdot| + c6 d_dipole rho_M |gdot| - c5 rho_SSD |gdot|
                   - c7 exp(-Q_bulk / kB T) (sigma_vm / kB T) rho_SSD^2 gdot_vm^c8,
  d_dipole = sqrt3 mu b / (16 pi (1 - nu) |tau|).

Readings where the paper is silent: the mobile density is Ma and Roters'
rho_M = 2 kB T / (c1 c2 c3 mu b^3) sqrt(rho_P rho_F) (the paper uses it
without a formula); nu_D = 1e13 /s ("in the order of the Debye frequency");
Poisson's ratio nu = 0.34 (copper); sigma_vm is the voxel's von Mises stress
and gdot_vm the von Mises equivalent plastic strain rate sqrt(2/3 epsdot_p:
epsdot_p); t = n x d (see oracle.gnd); the initial SSD density of a voxel is
split equally over the 12 systems; tau_pass, tau_cut and gdot_0 are frozen
during an increment (densities of its start) and the densities advance
explicitly from the converged slip rates, as for the power law.

Local potential: the flow rule is the derivative of the convex
psi(tau) = gdot_0 e^{-Q/kT} tau_cut (cosh((|tau| - tau_pass)/tau_cut) - 1)
above the threshold (0 below), so the local problem keeps its convex form.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .gnd import sense_vectors

KB = 1.380649e-23  # J/K


@dataclass(frozen=True)
class MaRoters:
    T: float = 473.0          # K (Sec. 3)
    Qslip: float = 3.3e-19    # J (Table 1)
    Qbulk: float = 3.51e-19   # J (Table 1)
    c1: float = 0.5
    c2: float = 3.0
    c3: float = 3.0
    c4: float = 8.0e7         # 1/m
    c5: float = 10.0
    c6: float = 3.0e10        # 1/m
    c7: float = 7.0e-28       # m^5 s^(c8-1)
    c8: float = 0.24
    nuD: float = 1.0e13       # 1/s (reading)
    poisson: float = 0.34     # (reading)
    mu: float = 47337.0       # MPa
    b: float = 2.56e-10       # m


def interaction_tables():
    """|cos| and |sin| of the angles (n^a, t^b) and (n^a, d^b), each (12, 12)."""
    n, d, t = sense_vectors()
    cnt = np.abs(n @ t.T)
    cnd = np.abs(n @ d.T)
    return cnt, np.sqrt(np.maximum(1.0 - cnt ** 2, 0.0)), cnd, np.sqrt(np.maximum(1.0 - cnd ** 2, 0.0))


def projections(rho_ssd, rho_gs=None, rho_get=None):
    """(rho_F, rho_P), each (V, 12), from per-system densities (V, 12)."""
    cnt, snt, cnd, snd = interaction_tables()
    F = rho_ssd @ cnt.T
    P = rho_ssd @ snt.T
    if rho_gs is not None:
        F = F + np.abs(rho_gs) @ cnd.T + np.abs(rho_get) @ cnt.T
        P = P + np.abs(rho_gs) @ snd.T + np.abs(rho_get) @ snt.T
    return F, P


def slip_parameters(law: MaRoters, rhoF, rhoP):
    """(tau_pass MPa, tau_cut MPa, A = gdot_0 exp(-Q/kT) 1/s), each (V, 12)."""
    kT = KB * law.T
    mu_pa = law.mu * 1e6
    tau_pass = law.c1 * law.mu * law.b * np.sqrt(rhoP)
    tau_cut = law.Qslip / (law.c2 * law.c3 * law.b ** 2) * np.sqrt(rhoF) * 1e-6
    gdot0 = 2.0 * kT / (law.c1 * law.c3 * mu_pa * law.b ** 2) * law.nuD * np.sqrt(rhoP)
    return tau_pass, tau_cut, gdot0 * np.exp(-law.Qslip / kT)


class MRFlow:
    """Flow of the 12 systems at frozen per-system parameters (V, 12)."""

    def __init__(self, tau_pass, tau_cut, A):
        self.tp, self.tc, self.A = tau_pass, tau_cut, A

    def sub(self, ix):
        return MRFlow(self.tp[ix], self.tc[ix], self.A[ix])

    def _x(self, tau):
        return (np.abs(tau) - self.tp) / self.tc

    def rate(self, tau):
        x = self._x(tau)
        with np.errstate(over="ignore"):
            return np.where(x > 0, self.A * np.sinh(np.maximum(x, 0.0)) * np.sign(tau), 0.0)

    def drate(self, tau):
        x = self._x(tau)
        with np.errstate(over="ignore"):
            return np.where(x > 0, self.A / self.tc * np.cosh(np.maximum(x, 0.0)), 0.0)

    def psi(self, tau):
        x = self._x(tau)
        with np.errstate(over="ignore"):
            return np.where(x > 0, self.A * self.tc * (np.cosh(np.maximum(x, 0.0)) - 1.0), 0.0)


def ssd_rates(law: MaRoters, rho_ssd, rhoF, rhoP, tau, gdot, sig_vm_mpa, gdot_vm):
    """rhodot_SSD (V, 12), Eq. 6."""
    kT = KB * law.T
    mu_pa = law.mu * 1e6
    ag = np.abs(gdot)
    rho_m = 2.0 * kT / (law.c1 * law.c2 * law.c3 * mu_pa * law.b ** 3) * np.sqrt(rhoP * rhoF)
    with np.errstate(divide="ignore", invalid="ignore"):
        d_dip = np.where(ag > 0, np.sqrt(3.0) * law.mu * law.b / (16.0 * np.pi * (1.0 - law.poisson)
                                                                  * np.abs(tau)), 0.0)
    climb = (law.c7 * np.exp(-law.Qbulk / kT) * (sig_vm_mpa[:, None] * 1e6 / kT) * rho_ssd ** 2
             * (gdot_vm[:, None] ** law.c8))
    return (law.c4 * np.sqrt(rhoF) * ag + law.c6 * d_dip * rho_m * ag - law.c5 * rho_ssd * ag - climb)


def von_mises_stress(sig_mandel):
    """sqrt(3/2 s':s') per voxel; sig (V, 6) Mandel."""
    dev = sig_mandel.copy()
    dev[:, :3] -= sig_mandel[:, :3].mean(axis=1, keepdims=True)
    return np.sqrt(1.5 * np.sum(dev * dev, axis=1))


def von_mises_rate(epsdot_mandel):
    """sqrt(2/3 e:e) per voxel of a (traceless) rate (V, 6) Mandel."""
    return np.sqrt(2.0 / 3.0 * np.sum(epsdot_mandel * epsdot_mandel, axis=1))
