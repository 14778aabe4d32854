"""Gradients of a volume-averaged stress-strain curve (reverse mode).

``StressStrainCurve.apply(theta, problem)`` runs the increments of a loading
path on the GPU and returns the curve <sigma33>_t, t = 1..T, as a tensor; its
backward pass gives d(loss)/d(theta) for theta = (tau0, k1, k2, n) through
the library's adjoint of each converged increment (implicit differentiation
of the fixed point, one linear tangent solve per increment).

Memory: the forward keeps a state snapshot every ``checkpoint_every``
increments, and after the last one; the backward recomputes one segment at a
time from its checkpoint (the segment's end is the next checkpoint, so k - 1
increments per segment of k), keeping that segment's snapshots, then walks it
in reverse. The default interval is the smallest whose snapshots fit in half
of the free device memory: every increment's state when they all fit (no
recomputation at all), else longer segments, at most ceil(sqrt T).
Recomputation is bit-identical because every kernel is deterministic, so
every schedule gives the same gradient.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np
import torch

from .fftevp import Load, Material, Opts, Solver, OK


@dataclass
class CurveProblem:
    solver: Solver
    material: Material
    quat: object
    rho: object
    load: Load
    increments: int
    opts: Opts = None
    adjoint_opts: Opts = None
    checkpoint_every: int = 0  # 0: the smallest interval that fits in memory (see the module notes)
    iterations: list = None   # fixed-point iterations of the latest forward, per increment
    schedule: int = 0         # checkpoint interval of the latest forward


def _material(base: Material, theta) -> Material:
    th = [float(x) for x in theta]
    return replace(base, tau0=th[0], k1=th[1], k2=th[2], n=th[3])


def _forward(p: CurveProblem, theta, keep_every):
    s = p.solver
    s.set_material(_material(p.material, theta))
    s.set_microstructure(p.quat, p.rho)
    s.set_loading(p.load)
    ckpts = {0: s.save_state()}
    curve = []
    p.iterations = []
    for t in range(1, p.increments + 1):
        r = s.step(p.opts)
        if r.status != OK:
            raise RuntimeError(f"increment {t} did not converge (status {r.status})")
        curve.append(r.Sigma[2])
        p.iterations.append(r.iters)
        if keep_every and (t % keep_every == 0 or t == p.increments):
            ckpts[t] = s.save_state()
    return np.array(curve), ckpts


def _schedule(p: CurveProblem) -> int:
    """Checkpoint interval k: the smallest with ceil(T / k) + 1 checkpoints
    plus the k - 1 recomputed states of one segment within half of the free
    device memory; ceil(sqrt T) when even that does not fit."""
    T = p.increments
    if p.checkpoint_every:
        return p.checkpoint_every
    k_max = max(1, int(math.ceil(math.sqrt(T))))
    snap = p.solver.state_bytes()
    free, _ = torch.cuda.mem_get_info()
    for k in range(1, k_max):
        if (math.ceil(T / k) + 1 + (k - 1)) * snap <= 0.5 * free:
            return k
    return k_max


def curve(p: CurveProblem, theta):
    """<sigma33>_t for t = 1..T (no gradient bookkeeping)."""
    c, _ = _forward(p, theta, 0)
    return c


class StressStrainCurve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, p: CurveProblem):
        every = _schedule(p)
        p.schedule = every
        c, ckpts = _forward(p, theta.detach().cpu().numpy(), every)
        ctx.p, ctx.every, ctx.ckpts = p, every, ckpts
        ctx.theta = theta.detach().cpu().numpy()
        return torch.as_tensor(c, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad):
        p, every, ckpts = ctx.p, ctx.every, ctx.ckpts
        s = p.solver
        # the solver may have run other parameters since this forward (several
        # curves in one loss, a line search): the recomputed segments and the
        # adjoint solves must use this forward's parameters, microstructure
        # and loading (snapshots hold the state, not these)
        s.set_material(_material(p.material, ctx.theta))
        s.set_microstructure(p.quat, p.rho)
        s.set_loading(p.load)
        g = grad.detach().cpu().numpy().astype(np.float64)
        T = p.increments
        adj = torch.zeros(s.adjoint_bytes(), dtype=torch.uint8, device="cuda")
        dth = np.zeros(4)
        starts = sorted(ckpts)
        for a in reversed(starts[:-1] if starts[-1] == T else starts):
            b = min(a + every, T)
            states = [ckpts[a]]
            if b - a > 1:
                s.load_state(ckpts[a])
            for t in range(a + 1, b + 1):
                if t in ckpts:      # the segment's end: stored by the forward
                    states.append(ckpts[t])
                    continue
                r = s.step(p.opts)
                if r.status != OK:
                    raise RuntimeError("recomputation did not converge")
                states.append(s.save_state())
            for t in range(b, a, -1):
                dS = (0.0, 0.0, float(g[t - 1]), 0.0, 0.0, 0.0)
                dth = s.adjoint_increment(states[t - 1 - a], states[t - a], dS, adj, dth,
                                          p.adjoint_opts or p.opts)
            del states
        return torch.as_tensor(dth, dtype=grad.dtype), None


def curve_loss(c, target):
    """L = (1/T) sum_t (<sigma33>_t - target_t)^2 (MPa^2)."""
    return torch.mean((c - target) ** 2)
