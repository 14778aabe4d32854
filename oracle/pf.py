"""Phase-field growth of recrystallised grains (Sec. 2.4, Eq. 12-15) —
TEST INFRASTRUCTURE ONLY.

Two order parameters per grain, eta_rex,i and eta_def,i (a deformed grain
has eta_def = 1, a recrystallised one eta_rex = 1). Free energy density:
the multi-well grain-boundary term of Eq. 13 with its gradient energy, and
the stored energy of Eq. 14, f_def = E_store D / S with D = sum eta_def^2,
S = sum (eta_rex^2 + eta_def^2), E_store = rho_tot zeta mu b^2. Allen-Cahn
(Eq. 15) for every order parameter eta_p:

    d eta_p / dt = -L [ m (eta_p^3 - eta_p + 3 eta_p sum_{q != p} eta_q^2)
                        - kappa lap(eta_p) + d f_def / d eta_p ],
    d f_def / d eta_rex,i = -2 E_store eta_rex,i D / S^2,
    d f_def / d eta_def,i =  2 E_store eta_def,i R / S^2,  R = sum eta_rex^2,

with m = 6 omega/l, kappa = 3 omega l / 4, L = 4 M / (3 l) (the coefficients
of Eq. 13 and 15).

Readings. Pair coefficient: as printed, Eq. 13 counts every (rex, def)
pair twice (once in each line) and every (rex, rex) or (def, def) pair once;
the coefficient relations it takes from the quantitative model hold for the
symmetric multi-well form with the same pair coefficient 3/2 on every pair,
which is the form used here (the derivative above). Units: the paper fixes the discretisation by 6 omega = l (in the
units of the quantitative scheme it cites), l = sqrt(9.6) dx and
M dt = 0.0375 l; the solver works in those units, grid spacing dx = 1 and
one PF step dt = 1, so l = sqrt(9.6), omega = l/6, M = 0.0375 l, i.e.
m = 1, kappa = 1.2, L = 0.05, and the energy density unit is 6 omega_SI /
l_SI with l_SI = sqrt(9.6) dx_SI: E_store enters as rho_tot zeta mu b^2 /
(6 omega_SI / l_SI). The real time of one PF step is 0.225 omega / M (the
formula stated in Sec. 2.4). Explicit Euler, 7-point Laplacian, periodic.
Sparse storage (the cited sparse-data technique): a grid point keeps at most
K order parameters, those above a threshold, largest first; an order
parameter absent from a point is zero there. Refinement 2:1 (Sec. 2.4): fine
point (2i + a) (a in {0, 1} per axis) takes the grain of coarse point i
(nearest grid point; the midpoints take the lower one) and E_store from
trilinear interpolation of the coarse points i and i + 1 (periodic); after
the PF steps coarse point i takes the grain of the largest order parameter
at fine point 2i (reading: a point that holds none keeps its grain). Order parameter keys: 2 id + kind (kind 1 = rex, 0 = def);
nuclei (negative ids) start recrystallised.

Arrays: dense order parameters (P, Vf) over an explicit key list; voxels
``[z][y][x]``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

L_GB = np.sqrt(9.6)
M_COEF = 1.0          # 6 omega / l in the solver's units
KAPPA = 9.6 / 8.0     # 3 omega l / 4 with omega = l / 6
L_KIN = 0.05          # 4 M / (3 l) with M = 0.0375 l


@dataclass(frozen=True)
class PF:
    omega: float = 0.625       # J/m^2 (Table 2)
    mobility: float = 145e-6   # m^4/(J s) (Table 2: 145 m^4/(MJ s))
    zeta: float = 0.25         # (Table 2)
    K: int = 6                 # order parameters kept per point
    threshold: float = 1e-5    # smaller values are dropped


def step_time(pf: PF):
    """Real time of one PF step, 0.225 omega / M (Sec. 2.4)."""
    return 0.225 * pf.omega / pf.mobility


def energy_unit(dx_si, pf: PF):
    return 6.0 * pf.omega / (L_GB * dx_si)


def refine_grain(grains_c, shape_c):
    """Coarse grain map (V,) -> fine (8V,), nearest (lower) coarse point."""
    n0, n1, n2 = shape_c
    g = np.asarray(grains_c).reshape(n2, n1, n0)
    return np.repeat(np.repeat(np.repeat(g, 2, axis=0), 2, axis=1), 2, axis=2).reshape(-1)


def refine_linear(f_c, shape_c):
    """Trilinear 2:1 prolongation of a coarse field (V,) -> (8V,), periodic."""
    n0, n1, n2 = shape_c
    f = np.asarray(f_c, dtype=np.float64).reshape(n2, n1, n0)
    for ax in (0, 1, 2):
        nxt = np.roll(f, -1, axis=ax)
        out = np.empty(f.shape[:ax] + (2 * f.shape[ax],) + f.shape[ax + 1:])
        sl0 = [slice(None)] * 3
        sl1 = [slice(None)] * 3
        sl0[ax] = slice(0, None, 2)
        sl1[ax] = slice(1, None, 2)
        out[tuple(sl0)] = f
        out[tuple(sl1)] = 0.5 * (f + nxt)
        f = out
    return f.reshape(-1)


def keys_of(grains):
    """Order-parameter key of each grain id: 2 id + 1 for nuclei (rex)."""
    g = np.asarray(grains, dtype=np.int64)
    return 2 * g + (g < 0)


def laplacian(a, shape_f):
    n0, n1, n2 = shape_f
    x = a.reshape(a.shape[0], n2, n1, n0)
    lap = -6.0 * x
    for ax in (1, 2, 3):
        lap = lap + np.roll(x, 1, axis=ax) + np.roll(x, -1, axis=ax)
    return lap.reshape(a.shape)


def truncate(eta, K, thr):
    """Keep, per point, the K largest values above thr (others zero)."""
    out = np.where(eta > thr, eta, 0.0)
    if out.shape[0] > K:
        order = np.argsort(-out, axis=0, kind="stable")
        drop = order[K:]
        np.put_along_axis(out, drop, 0.0, axis=0)
    return out


def pf_step(eta, is_rex, E, shape_f, pf: PF):
    """One explicit step of all order parameters (P, Vf); is_rex (P,) bool."""
    s2 = (eta ** 2).sum(axis=0)
    R = (eta[is_rex] ** 2).sum(axis=0)
    D = (eta[~is_rex] ** 2).sum(axis=0)
    S = R + D
    with np.errstate(divide="ignore", invalid="ignore"):
        dfr = np.where(S > 0, -2.0 * E * D / S ** 2, 0.0)
        dfd = np.where(S > 0, 2.0 * E * R / S ** 2, 0.0)
    dfdef = np.where(is_rex[:, None], dfr[None] * eta, dfd[None] * eta)
    dF = M_COEF * (eta ** 3 - eta + 3.0 * eta * (s2[None] - eta ** 2)) - KAPPA * laplacian(eta, shape_f) + dfdef
    return truncate(eta - L_KIN * dF, pf.K, pf.threshold)


def initial_state(grains_c, shape_c):
    """(keys (P,), dense eta (P, 8V)) on the fine grid from the coarse grain map."""
    gf = refine_grain(grains_c, shape_c)
    kf = keys_of(gf)
    keys = np.unique(kf)
    eta = (kf[None, :] == keys[:, None]).astype(np.float64)
    return keys, eta


def coarse_grains(keys, eta, shape_c, grains_before):
    """Grain of the largest order parameter at fine point 2i, per coarse i
    (equal values: the smaller key); a point holding none keeps its grain."""
    n0, n1, n2 = shape_c
    e = eta.reshape(len(keys), 2 * n2, 2 * n1, 2 * n0)[:, ::2, ::2, ::2].reshape(len(keys), -1)
    k = keys[np.argmax(e, axis=0)]
    return np.where(e.max(axis=0) > 0, np.floor_divide(k, 2), np.asarray(grains_before).reshape(-1))
