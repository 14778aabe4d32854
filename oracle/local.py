"""Per-voxel constitutive solve of the oracle (test infrastructure only).

Flow rule: power law on the resolved shear of each slip system,
``gdot_a = gdot0 * |tau_a / tauc|^n * sign(tau_a)`` with ``tau_a = m_a : sigma``,
one critical resolved shear stress ``tauc`` per voxel.
Plastic strain rate: ``epsdot_p = sum_a m_a gdot_a`` (Eq. 2).

Implicit Euler Hooke law (Eq. 1) with the augmented-Lagrangian penalty
(Sec. 2.1, the nonlinear local equations are solved with an augmented
Lagrangian scheme): for given multiplier ``lam`` and compatible strain
``e`` the local stress minimises the strictly convex potential

    Phi(s) = 1/2 (s-lam):C0^-1:(s-lam) + 1/2 s:S:s + s:(epsp - e)
             + dt * sum_a gdot0 * tauc / (n+1) * |tau_a / tauc|^(n+1)

whose stationarity is ``C0^-1:(s-lam) + S:s + epsp + dt*epsdot_p(s) - e = 0``.
The oracle minimises Phi by Newton's method with a backtracking line search,
all in FP64, in the sample frame, voxel by voxel (vectorised over voxels).
"""
from __future__ import annotations

import numpy as np


def resolved_shear(sig, m):
    """tau_a = m_a : sigma; sig (M,6) Mandel, m (M,12,6) -> (M,12)."""
    return (m @ sig[:, :, None])[:, :, 0]


def slip_rates(sig, m, tauc, gdot0, n):
    """(tau, gdot) for each voxel and slip system."""
    tau = resolved_shear(sig, m)
    x = tau / tauc[:, None]
    gdot = gdot0 * np.abs(x) ** n * np.sign(x)
    return tau, gdot


def plastic_rate(sig, m, tauc, gdot0, n):
    """epsdot_p = sum_a m_a gdot_a (Eq. 2), Mandel (M, 6)."""
    _, gdot = slip_rates(sig, m, tauc, gdot0, n)
    return (gdot[:, None, :] @ m)[:, 0, :]


def potential(sig, lam, e, epsp, S, C0inv, m, tauc, gdot0, n, dt):
    d = sig - lam
    tau = resolved_shear(sig, m)
    x = np.abs(tau / tauc[:, None])
    visc = (gdot0 * tauc[:, None] / (n + 1.0) * x ** (n + 1.0)).sum(axis=1)
    Ss = (S @ sig[:, :, None])[:, :, 0]
    return (0.5 * np.sum(d * (d @ C0inv.T), axis=1)
            + 0.5 * np.sum(sig * Ss, axis=1)
            + np.sum(sig * (epsp - e), axis=1)
            + dt * visc)


def residual(sig, lam, e, epsp, S, C0inv, m, tauc, gdot0, n, dt):
    return ((sig - lam) @ C0inv.T + (S @ sig[:, :, None])[:, :, 0] + epsp
            + dt * plastic_rate(sig, m, tauc, gdot0, n) - e)


def jacobian(sig, S, C0inv, m, tauc, gdot0, n, dt):
    """d residual / d sigma = C0^-1 + S + dt * sum_a dgdot_a/dtau_a m_a m_a^T."""
    tau = resolved_shear(sig, m)
    x = np.abs(tau / tauc[:, None])
    dg = gdot0 * n * x ** (n - 1.0) / tauc[:, None]
    mt = np.swapaxes(m, 1, 2) * dg[:, None, :]
    return C0inv[None] + S + dt * (mt @ m)


def local_solve(lam, e, epsp, tauc, S, m, C0inv, gdot0, n, dt, sig0=None,
                tol=1e-12, max_iter=100):
    """Minimise Phi voxel by voxel. All tensors Mandel, shape (M, 6).

    Stops a voxel once the Newton step satisfies
    ``|step| <= tol * max(|sigma|, 1 MPa)``. Returns (sigma, iterations,
    number of voxels that did not converge).
    """
    sig = np.array(lam if sig0 is None else sig0, dtype=np.float64, copy=True)
    M = sig.shape[0]
    active = np.ones(M, dtype=bool)
    iters = np.zeros(M, dtype=np.int64)
    args = lambda ix: (lam[ix], e[ix], epsp[ix], S[ix], C0inv, m[ix], tauc[ix])
    for _ in range(max_iter):
        ix = np.flatnonzero(active)
        if ix.size == 0:
            break
        l_, e_, p_, S_, C_, m_, t_ = args(ix)
        s = sig[ix]
        r = residual(s, l_, e_, p_, S_, C_, m_, t_, gdot0, n, dt)
        J = jacobian(s, S_, C_, m_, t_, gdot0, n, dt)
        step = -np.linalg.solve(J, r[..., None])[..., 0]
        f0 = potential(s, l_, e_, p_, S_, C_, m_, t_, gdot0, n, dt)
        slope = np.einsum("mk,mk->m", r, step)
        rn0 = np.linalg.norm(r, axis=1)
        t = np.ones(ix.size)
        todo = np.ones(ix.size, dtype=bool)
        for _ls in range(60):
            k = np.flatnonzero(todo)
            if k.size == 0:
                break
            cand = s[k] + t[k, None] * step[k]
            with np.errstate(over="ignore", invalid="ignore"):
                f1 = potential(cand, l_[k], e_[k], p_[k], S_[k], C_, m_[k], t_[k],
                               gdot0, n, dt)
                r1 = residual(cand, l_[k], e_[k], p_[k], S_[k], C_, m_[k], t_[k],
                              gdot0, n, dt)
            ok = np.isfinite(f1) & ((f1 <= f0[k] + 1e-4 * t[k] * slope[k])
                                    | (np.linalg.norm(r1, axis=1) <= 0.5 * rn0[k]))
            todo[k[ok]] = False
            t[k[~ok]] *= 0.5
        dx = t[:, None] * step
        s_new = s + dx
        sig[ix] = s_new
        iters[ix] += 1
        scale = np.maximum(np.linalg.norm(s_new, axis=1), 1.0)
        done = np.linalg.norm(dx, axis=1) <= tol * scale
        active[ix[done]] = False
    return sig, iters, int(active.sum())


def constitutive_strain(sig, epsp, S, m, tauc, gdot0, n, dt):
    """eps = S:sigma + epsp + dt * epsdot_p(sigma)   (Eq. 1 rearranged)."""
    return ((S @ sig[:, :, None])[:, :, 0] + epsp
            + dt * plastic_rate(sig, m, tauc, gdot0, n))


# ---- general flow rule (per-system rate, its derivative and its potential) --
# Same minimisation for any flow object with rate(tau), drate(tau), psi(tau)
# on (M, 12) resolved shears and sub(ix) restricting it to voxels ix; the
# power law above is the special case psi = gdot0 tauc/(n+1) |tau/tauc|^(n+1).

def plastic_rate_flow(sig, m, flow):
    gd = flow.rate(resolved_shear(sig, m))
    return (gd[:, None, :] @ m)[:, 0, :]


def potential_flow(sig, lam, e, epsp, S, C0inv, m, flow, dt):
    d = sig - lam
    Ss = (S @ sig[:, :, None])[:, :, 0]
    return (0.5 * np.sum(d * (d @ C0inv.T), axis=1) + 0.5 * np.sum(sig * Ss, axis=1)
            + np.sum(sig * (epsp - e), axis=1) + dt * flow.psi(resolved_shear(sig, m)).sum(axis=1))


def residual_flow(sig, lam, e, epsp, S, C0inv, m, flow, dt):
    return ((sig - lam) @ C0inv.T + (S @ sig[:, :, None])[:, :, 0] + epsp
            + dt * plastic_rate_flow(sig, m, flow) - e)


def jacobian_flow(sig, S, C0inv, m, flow, dt):
    dg = flow.drate(resolved_shear(sig, m))
    mt = np.swapaxes(m, 1, 2) * dg[:, None, :]
    return C0inv[None] + S + dt * (mt @ m)


def local_solve_flow(lam, e, epsp, S, m, C0inv, flow, dt, sig0=None, tol=1e-12, max_iter=100):
    """Minimise Phi with a general flow rule; same Newton iteration, line
    search and stop rule as ``local_solve``."""
    sig = np.array(lam if sig0 is None else sig0, dtype=np.float64, copy=True)
    M = sig.shape[0]
    active = np.ones(M, dtype=bool)
    iters = np.zeros(M, dtype=np.int64)
    for _ in range(max_iter):
        ix = np.flatnonzero(active)
        if ix.size == 0:
            break
        l_, e_, p_, S_, m_, f_ = lam[ix], e[ix], epsp[ix], S[ix], m[ix], flow.sub(ix)
        s = sig[ix]
        r = residual_flow(s, l_, e_, p_, S_, C0inv, m_, f_, dt)
        J = jacobian_flow(s, S_, C0inv, m_, f_, dt)
        step = -np.linalg.solve(J, r[..., None])[..., 0]
        f0 = potential_flow(s, l_, e_, p_, S_, C0inv, m_, f_, dt)
        slope = np.einsum("mk,mk->m", r, step)
        rn0 = np.linalg.norm(r, axis=1)
        t = np.ones(ix.size)
        todo = np.ones(ix.size, dtype=bool)
        for _ls in range(60):
            k = np.flatnonzero(todo)
            if k.size == 0:
                break
            cand = s[k] + t[k, None] * step[k]
            fk = f_.sub(k)
            with np.errstate(over="ignore", invalid="ignore"):
                f1 = potential_flow(cand, l_[k], e_[k], p_[k], S_[k], C0inv, m_[k], fk, dt)
                r1 = residual_flow(cand, l_[k], e_[k], p_[k], S_[k], C0inv, m_[k], fk, dt)
            ok = np.isfinite(f1) & ((f1 <= f0[k] + 1e-4 * t[k] * slope[k])
                                    | (np.linalg.norm(r1, axis=1) <= 0.5 * rn0[k]))
            todo[k[ok]] = False
            t[k[~ok]] *= 0.5
        dx = t[:, None] * step
        s_new = s + dx
        sig[ix] = s_new
        iters[ix] += 1
        scale = np.maximum(np.linalg.norm(s_new, axis=1), 1.0)
        done = np.linalg.norm(dx, axis=1) <= tol * scale
        active[ix[done]] = False
    return sig, iters, int(active.sum())


def constitutive_strain_flow(sig, epsp, S, m, flow, dt):
    return (S @ sig[:, :, None])[:, :, 0] + epsp + dt * plastic_rate_flow(sig, m, flow)
