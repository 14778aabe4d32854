"""FFT-EVP fixed-point solve of the oracle (test infrastructure only).

One strain increment t -> t+dt (Sec. 2.1, Eq. 1-2; augmented Lagrangian of
the nonlinear local equations, Sec. 2.1), written step by step:

    E <- E_t with the strain-controlled components advanced by Edot*dt
    e <- e_t + (E - E_t);  lam <- sigma_t
    repeat:
      (1) sigma = argmin Phi per voxel (local.local_solve);
          eps = S:sigma + epsp_t + dt*epsdot_p(sigma)
      (2) err_c  = rms|e - eps| / |E|
          err_bc = |(Sigma* - <sigma>)_s| / |<sigma>|    (s: stress-controlled)
          stop when both are below tol
      (3) E_s += [(C0)_ss]^-1 (Sigma* - <sigma>)_s
      (4) tau = sigma - C0:eps ; tau_hat = FFT(tau)
      (5) e_hat = -Gamma0:tau_hat (C0^-1 at Nyquist), e_hat(0) = N^3 E;
          e = IFFT(e_hat); lam = sigma
    state update: epsp += dt*epsdot_p(sigma);
                  rho  += dt*(k1 sqrt(rho) - k2 rho) * sum_a |gdot_a(sigma)|
                  tauc  = tau0 + alpha*mu*b*sqrt(rho)

The hardening law is a Kocks-Mecking storage/recovery law on one density
per voxel; its storage and athermal-recovery terms play the roles of the
lock-forming (c4) and athermal-annihilation (c5) terms of the SSD evolution
(Sec. 2.2, Eq. 6), and the Taylor constant that of c1 in the passing stress
(Sec. 2.2, Eq. 3). The plastic strain follows the first-order update stated
after Eq. 1.

Units: MPa, s, m, m^-2. Public arrays are plain components
[11, 22, 33, 23, 13, 12], component-major, voxels ``[z][y][x]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from . import local as L
from .crystal import voxel_material
from . import drx as DX
from . import ma_roters as MR
from . import pf as PF
from . import rotation as ROT
from .gnd import gnd_rates, next_leff
from .green import gamma_field, green_apply
from .tensors import (isotropic_c4, mandel_to_voigt, voigt_to_mandel, c4_to_mandel)

# cubic Cu elastic constants (MPa)
CU = dict(C11=168400.0, C12=121400.0, C44=75400.0)


@dataclass
class Flow:
    tau0: float = 5.0          # MPa
    k1: float = 8.0e7          # 1/m
    k2: float = 10.0           # -
    n: float = 10.0            # rate exponent
    gdot0: float = 1.0e-3      # 1/s
    alpha: float = 0.5         # Taylor constant
    mu: float = 47337.0        # MPa (Hill average shear modulus of Cu)
    b: float = 2.56e-10        # m

    def theta(self):
        return np.array([self.tau0, self.k1, self.k2, self.n])

    def with_theta(self, th):
        return replace(self, tau0=float(th[0]), k1=float(th[1]), k2=float(th[2]),
                       n=float(th[3]))


@dataclass
class Loading:
    Edot: np.ndarray = field(default_factory=lambda: np.array([0, 0, -1e-3, 0, 0, 0.0]))
    Sigma: np.ndarray = field(default_factory=lambda: np.zeros(6))
    strain_ctrl: np.ndarray = field(default_factory=lambda: np.array([0, 0, 1, 0, 0, 0]))
    dt: float = 2.0


def default_c0(C11, C12, C44):
    """Isotropic reference medium (lambda0, mu0): the crystal's bulk modulus and
    1/16 of its Voigt-average shear modulus. The converged fields do not depend
    on this choice; a shear modulus between the elastic and the viscoplastic
    tangent moduli makes the iteration converge in tens of steps."""
    K = (C11 + 2 * C12) / 3.0
    mu = (C11 - C12 + 3 * C44) / 5.0 / 16.0
    return K - 2.0 * mu / 3.0, mu


class Oracle:
    """Plain FP64 CPU implementation of the increment loop."""

    def __init__(self, shape, quat, rho, C11=CU["C11"], C12=CU["C12"], C44=CU["C44"],
                 flow: Flow | None = None, c0=None, plastic=True):
        self.shape = tuple(int(s) for s in shape)
        self.nvox = int(np.prod(self.shape))
        self.flow = flow or Flow()
        self.plastic = plastic
        self.elastic = (C11, C12, C44)
        self.quat = np.asarray(quat, dtype=np.float64).reshape(4, -1).copy()
        self.C, self.S, self.m = voxel_material(quat, C11, C12, C44)
        self.gnd = None
        self.mr = None
        self.rot = False
        lam0, mu0 = c0 if c0 is not None else default_c0(C11, C12, C44)
        self.c0 = (lam0, mu0)
        self.C0_4 = isotropic_c4(lam0, mu0)
        self.C0 = c4_to_mandel(self.C0_4)
        self.C0inv = np.linalg.inv(self.C0)
        self.rho = np.asarray(rho, dtype=np.float64).reshape(-1).copy()
        self.epsp = np.zeros((self.nvox, 6))
        self.sigma = np.zeros((self.nvox, 6))
        self.e = np.zeros((self.nvox, 6))
        self.E = np.zeros(6)
        self.t = 0.0
        self._G = None

    def enable_gnd(self, grains, l0, xi):
        """Track GND densities (Sec. 2.2, Eq. 7-8; see oracle.gnd) from now on."""
        self.gnd = dict(grains=np.asarray(grains).reshape(-1).copy(), leff=float(l0), xi=float(xi),
                        rs=np.zeros((12, self.nvox)), ret=np.zeros((12, self.nvox)))

    def enable_drx(self, drx, u0):
        """DRX nucleation (Sec. 2.3, 2.5; see oracle.drx): draw the nucleation
        strengths from uniforms u0 (V,). Needs GND tracking (grain ids)."""
        assert self.gnd is not None, "DRX nucleation needs the grain ids of GND tracking"
        self.drx = drx
        self.kappa = DX.weibull_strength(u0, drx.kc, drx.q)

    def drx_nucleate(self, u):
        """Test every grain-boundary voxel on the current state; returns the
        number of new nuclei. u: fresh uniforms (V,) for the redraws."""
        G = self.gnd
        k = DX.total_density(self.rho, G["rs"], G["ret"], self.mr,
                             None if self.mr is None else self.ssd)
        sites = DX.gb_sites(G["grains"], self.shape)
        hit, self.kappa = DX.nucleate(self.kappa, k, sites, np.asarray(u, dtype=np.float64), self.drx)
        G["grains"] = np.where(hit, -(np.arange(self.nvox) + 1), G["grains"])
        G["rs"] = np.where(hit[None], self.drx.s_soften * G["rs"], G["rs"])
        G["ret"] = np.where(hit[None], self.drx.s_soften * G["ret"], G["ret"])
        return int(hit.sum())

    def drx_grow(self, nsteps, zeta, omega_gb, dx, K=6, threshold=1e-5):
        """Grain growth after nucleation (Sec. 2.4-2.5, see oracle.pf): stored
        energy rho_tot zeta mu b^2 in units of 6 omega / (sqrt(9.6) dx), PF
        steps on the 2:1 grid, grain map read back; voxels now in a
        recrystallised grain they did not belong to keep s_soften of their
        GND densities (Eq. 16; reading: they are points of a new grain).
        Returns (changed, now recrystallised) voxel counts."""
        G = self.gnd
        k = DX.total_density(self.rho, G["rs"], G["ret"], self.mr,
                             None if self.mr is None else self.ssd)
        unit = 6.0 * omega_gb / (np.sqrt(9.6) * dx)
        E = k * zeta * self.flow.mu * 1e6 * self.flow.b ** 2 / unit
        keys, eta = PF.initial_state(G["grains"], self.shape)
        Ef = PF.refine_linear(E, self.shape)
        is_rex = (keys & 1) == 1
        cfg = PF.PF(omega=omega_gb, zeta=zeta, K=K, threshold=threshold)
        fine = tuple(2 * s for s in self.shape)
        for _ in range(nsteps):
            eta = PF.pf_step(eta, is_rex, Ef, fine, cfg)
        new = PF.coarse_grains(keys, eta, self.shape, G["grains"])
        changed = new != G["grains"]
        soft = changed & (new < 0)
        G["rs"] = np.where(soft[None], self.drx.s_soften * G["rs"], G["rs"])
        G["ret"] = np.where(soft[None], self.drx.s_soften * G["ret"], G["ret"])
        G["grains"] = new
        return int(changed.sum()), int(soft.sum())

    def enable_rotation(self):
        """Rotate the lattice by its spin (oracle.rotation) after every
        increment from now on."""
        self.rot = True

    def enable_mr(self, law=None):
        """Use the paper's own flow rule and SSD evolution (Sec. 2.2, Eq. 3-6;
        see oracle.ma_roters) from now on; each voxel's density is split
        equally over the 12 systems."""
        self.mr = law or MR.MaRoters()
        self.ssd = np.repeat(self.rho[:, None] / 12.0, 12, axis=1)

    def mr_flow(self):
        G = self.gnd
        F, P = MR.projections(self.ssd, None if G is None else G["rs"].T,
                              None if G is None else G["ret"].T)
        return MR.MRFlow(*MR.slip_parameters(self.mr, F, P)), F, P

    # -- helpers ----------------------------------------------------------
    def tauc(self, rho=None, flow=None):
        f = flow or self.flow
        r = self.rho if rho is None else rho
        return f.tau0 + f.alpha * f.mu * f.b * np.sqrt(r)

    def _gdot0(self):
        return self.flow.gdot0 if self.plastic else 0.0

    def local(self, lam, e, tauc, sig0=None, tol=1e-12):
        f = self.flow
        return L.local_solve(lam, e, self.epsp, tauc, self.S, self.m, self.C0inv,
                             self._gdot0(), f.n, self._dt, sig0=sig0, tol=tol)

    def strain(self, sig, tauc):
        return L.constitutive_strain(sig, self.epsp, self.S, self.m, tauc,
                                     self._gdot0(), self.flow.n, self._dt)

    def spectral_update(self, tau, E):
        """(4)-(5): compatible strain from the polarisation field (Mandel (M,6))."""
        n0, n1, n2 = self.shape
        t = tau.T.reshape(6, n2, n1, n0)
        th = np.fft.fftn(t, axes=(1, 2, 3))
        if self._G is None:
            self._G = gamma_field(self.shape, self.C0_4, self.C0inv)
        eh = green_apply(th, self._G, E)
        e = np.fft.ifftn(eh, axes=(1, 2, 3))
        return np.ascontiguousarray(e.real.reshape(6, -1).T)

    # -- stress redistribution after the microstructure update -----------
    def mechanical_state(self):
        """Copy of the mechanical state (plastic strain, stress, compatible
        strain, mean strain) that a stress redistribution restarts from."""
        return dict(epsp=self.epsp.copy(), sigma=self.sigma.copy(), e=self.e.copy(), E=self.E.copy())

    def redistribute(self, before, load: Loading, tol=1e-6, max_iter=1000):
        """Stress redistribution (Sec. 2.5): after nucleation and growth have
        changed the microstructure, the equilibrium stress is computed again
        before further loading, with the strain rate of the last increment
        prescribed. Reading: the last increment's solve is repeated from its
        mechanical start state ``before`` (taken with mechanical_state() before
        that increment) with the same loading, i.e. the same prescribed
        macroscopic strain increment, and the current microstructure (the
        densities as the increment and the DRX update left them, so the slip
        resistances of the softened nuclei); the new stress, compatible and
        mean strain and the plastic strain of the repeated increment replace
        the old ones. Densities, grains, orientations and time stay."""
        self.epsp = before["epsp"].copy()
        self.sigma = before["sigma"].copy()
        self.e = before["e"].copy()
        self.E = before["E"].copy()
        return self.increment(load, tol=tol, max_iter=max_iter, mechanics_only=True)

    # -- one increment ----------------------------------------------------
    def increment(self, load: Loading, tol=1e-6, max_iter=1000, history=False, mechanics_only=False):
        """One strain increment. mechanics_only: advance only the stress,
        strain and plastic strain (the repeated solve of a redistribution):
        densities, GND densities, orientations and time are not updated."""
        self._dt = load.dt
        sc = np.asarray(load.strain_ctrl).astype(bool)
        s = ~sc
        Sig_star = voigt_to_mandel(np.asarray(load.Sigma, dtype=np.float64))
        E = self.E.copy()
        E[sc] += voigt_to_mandel(np.asarray(load.Edot, dtype=np.float64))[sc] * load.dt
        e = self.e + (E - self.E)[None, :]
        lam = self.sigma.copy()
        tauc = self.tauc()
        if self.mr is not None:
            mflow, rF, rP = self.mr_flow()
        C0ss_inv = np.linalg.inv(self.C0[np.ix_(s, s)]) if s.any() else None
        hist = []
        converged = False
        for it in range(max_iter):
            if self.mr is None:
                sig, nit, nfail = self.local(lam, e, tauc)
                eps = self.strain(sig, tauc)
            else:
                sig, nit, nfail = L.local_solve_flow(lam, e, self.epsp, self.S, self.m, self.C0inv,
                                                     mflow, self._dt)
                eps = L.constitutive_strain_flow(sig, self.epsp, self.S, self.m, mflow, self._dt)
            err_c = np.sqrt(np.mean(np.sum((e - eps) ** 2, axis=1))) / np.linalg.norm(E)
            Sm = sig.mean(axis=0)
            dS = (Sig_star - Sm)[s]
            nS = np.linalg.norm(Sm)
            nb = np.linalg.norm(dS)
            err_bc = nb / nS if nS > 0 else (0.0 if nb == 0 else np.inf)
            if history:
                hist.append(dict(err_c=err_c, err_bc=err_bc, newton_max=int(nit.max()),
                                 Sigma=mandel_to_voigt(Sm)))
            if err_c < tol and err_bc < tol:
                converged = True
                break
            if s.any():
                E[s] += C0ss_inv @ dS
            tau = sig - eps @ self.C0.T
            e = self.spectral_update(tau, E)
            lam = sig
        iters = it + 1
        # state update at the converged stress, density from the increment start
        f = self.flow
        if self.mr is None:
            _, gdot = L.slip_rates(sig, self.m, tauc, self._gdot0(), f.n)
            self.epsp = self.epsp + load.dt * np.einsum("ma,mak->mk", gdot, self.m)
            gsum = np.abs(gdot).sum(axis=1)
            if not mechanics_only:
                self.rho = self.rho + load.dt * (f.k1 * np.sqrt(self.rho) - f.k2 * self.rho) * gsum
        else:
            tau_a = L.resolved_shear(sig, self.m)
            gdot = mflow.rate(tau_a)
            epdot = np.einsum("ma,mak->mk", gdot, self.m)
            self.epsp = self.epsp + load.dt * epdot
            if not mechanics_only:
                self.ssd = self.ssd + load.dt * MR.ssd_rates(self.mr, self.ssd, rF, rP, tau_a, gdot,
                                                             MR.von_mises_stress(sig), MR.von_mises_rate(epdot))
                self.rho = self.ssd.sum(axis=1)
        e_start = self.e
        self.sigma, self.e, self.E = sig, e, E
        if mechanics_only:
            return dict(iters=iters, converged=converged, err_c=err_c, err_bc=err_bc,
                        Sigma=mandel_to_voigt(sig.mean(axis=0)), E=mandel_to_voigt(E),
                        rho_mean=float(self.rho.mean()), newton_fail=nfail)
        if self.gnd is not None:
            G = self.gnd
            rs, ret = gnd_rates(gdot.T, self.quat, G["grains"], self.shape, f.b, G["leff"])
            G["rs"] = G["rs"] + load.dt * rs
            G["ret"] = G["ret"] + load.dt * ret
            G["leff"] = next_leff(G["leff"], E, G["xi"])
        if self.rot:
            # lattice rotation from the local rotation of the increment's strain
            # change and its slip rates (oracle.rotation), after the GND update,
            # which uses the orientation they acted in
            dw = ROT.local_rotation(e - e_start, self.shape)
            self.quat = ROT.rotate(self.quat, gdot, load.dt, dw)
            self.C, self.S, self.m = voxel_material(self.quat, *self.elastic)
        self.t += load.dt
        rep = dict(iters=iters, converged=converged, err_c=err_c, err_bc=err_bc,
                   Sigma=mandel_to_voigt(sig.mean(axis=0)), E=mandel_to_voigt(E),
                   rho_mean=float(self.rho.mean()), newton_fail=nfail)
        if history:
            rep["history"] = hist
        return rep

    # -- public views (plain components, component-major) -----------------
    def field(self, name):
        a = {"sigma": self.sigma, "strain": self.e, "epsp": self.epsp}.get(name)
        if a is not None:
            return mandel_to_voigt(a.T)
        if name == "rho":
            return self.rho.copy()
        if name == "quat":
            return self.quat.copy()
        if name == "kappa":
            return self.kappa.copy()
        if name == "grain":
            return self.gnd["grains"].astype(np.float64)
        if name == "rho_ssd":
            return self.ssd.T.copy()
        if name in ("rho_gnds", "rho_gndet"):
            return self.gnd["rs" if name == "rho_gnds" else "ret"].copy()
        if name == "gdot":
            # flow rule (power law of reading R1, or Eq. 3 with the paper's law)
            # at the committed stress and the current densities, [12][V]
            if self.mr is not None:
                return self.mr_flow()[0].rate(L.resolved_shear(self.sigma, self.m)).T.copy()
            _, g = L.slip_rates(self.sigma, self.m, self.tauc(), self._gdot0(), self.flow.n)
            return g.T.copy()
        raise KeyError(name)


def run_path(oracle: Oracle, load: Loading, increments: int, tol=1e-6, max_iter=1000):
    """Run ``increments`` increments; returns the list of reports."""
    return [oracle.increment(load, tol=tol, max_iter=max_iter) for _ in range(increments)]


def curve_loss(s33, target):
    """L = (1/T) sum_t (<sigma33>_t - target_t)^2, stress in MPa."""
    s33 = np.asarray(s33)
    return float(np.mean((s33 - np.asarray(target)) ** 2))


def stress_curve(shape, quat, rho, flow: Flow, load: Loading, increments, tol=1e-13,
                 max_iter=5000, c0=None):
    """<sigma33>_t for t = 1..T from a fresh state."""
    o = Oracle(shape, quat, rho, flow=flow, c0=c0)
    reps = run_path(o, load, increments, tol=tol, max_iter=max_iter)
    return np.array([r["Sigma"][2] for r in reps]), reps


def fd_gradient(shape, quat, rho, flow: Flow, load: Loading, increments, target,
                rel_step=1e-5, tol=1e-13, c0=None):
    """Central finite differences of the curve loss w.r.t. (tau0, k1, k2, n)."""
    th = flow.theta()
    g = np.zeros(4)
    for k in range(4):
        h = rel_step * abs(th[k])
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        sp, _ = stress_curve(shape, quat, rho, flow.with_theta(tp), load, increments, tol, c0=c0)
        sm, _ = stress_curve(shape, quat, rho, flow.with_theta(tm), load, increments, tol, c0=c0)
        g[k] = (curve_loss(sp, target) - curve_loss(sm, target)) / (2 * h)
    return g
