"""Pins of the oracle's stress-strain curve, curve loss and finite-difference
gradient (the references of the adjoint), and of the time discretisation.

A uniform single crystal in the cube orientation under uniaxial compression
along [001] with stress-free lateral faces carries a uniform uniaxial stress
sigma33. By the cubic symmetry eight of the twelve systems are loaded at
Schmid factor 1/sqrt6 and the other four not at all, so the whole increment
of the oracle (implicit Hooke law of Eq. 1, plastic rate of Eq. 2 summed over
the systems, density updated explicitly after convergence) collapses to one
scalar equation per increment,

    sigma/E001 + p_t + dt (8/sqrt6) gdot0 |sigma/(sqrt6 tauc)|^n sign(sigma) = E33_t,
    p_{t+1}   = p_t + dt (8/sqrt6) gdot0 |sigma/(sqrt6 tauc)|^n sign(sigma),
    rho_{t+1} = rho_t + dt (k1 sqrt(rho_t) - k2 rho_t) 8 gdot0 |sigma/(sqrt6 tauc)|^n,

with E001 the [001] Young's modulus (1/S11 of the cubic compliance) and
tauc = tau0 + alpha mu b sqrt(rho_t). This scalar recursion shares no code
with the oracle (no fields, no FFT, no tensors). Run in forward-mode dual
numbers it gives the exact derivative of every sigma33_t, hence of the curve
loss, with respect to (tau0, k1, k2, n). It pins:

* ``stress_curve``: the oracle's curve equals the recursion at every increment;
* ``fd_gradient``: central differences of the oracle's loss equal the exact
  gradient in all four components (a swapped component or a wrong step fails);
* the Taylor test L(theta + h v) - L(theta) - h g.v = O(h^2);
* the recursion itself, against the closed-form steady state
  |sigma33| = sqrt6 tauc (sqrt6 |Edot| / (8 gdot0))^(1/n) and its derivatives
  with respect to tau0 and n.

Also here: halving the strain increment changes the curve by O(increment)
(first-order time discretisation of the density update).
"""
import math

import numpy as np
import pytest

import synth
from oracle import Flow, Loading, CU, stress_curve, fd_gradient, curve_loss, Oracle

C11, C12, C44 = CU["C11"], CU["C12"], CU["C44"]


class Dual:
    """a + sum_k d_k eps_k with eps_k eps_l = 0 (forward-mode derivatives)."""

    def __init__(self, a, d=None, nd=4):
        self.a = float(a)
        self.d = np.zeros(nd) if d is None else np.asarray(d, dtype=float)

    @staticmethod
    def lift(x, nd):
        return x if isinstance(x, Dual) else Dual(x, None, nd)

    def __add__(self, o):
        o = Dual.lift(o, len(self.d))
        return Dual(self.a + o.a, self.d + o.d)

    __radd__ = __add__

    def __neg__(self):
        return Dual(-self.a, -self.d)

    def __sub__(self, o):
        return self + (-Dual.lift(o, len(self.d)))

    def __rsub__(self, o):
        return Dual.lift(o, len(self.d)) - self

    def __mul__(self, o):
        o = Dual.lift(o, len(self.d))
        return Dual(self.a * o.a, self.a * o.d + o.a * self.d)

    __rmul__ = __mul__

    def __truediv__(self, o):
        o = Dual.lift(o, len(self.d))
        return Dual(self.a / o.a, (self.d * o.a - self.a * o.d) / (o.a * o.a))

    def __rtruediv__(self, o):
        return Dual.lift(o, len(self.d)) / self


def dlog(x):
    return Dual(math.log(x.a), x.d / x.a)


def dexp(x):
    e = math.exp(x.a)
    return Dual(e, e * x.d)


def dsqrt(x):
    r = math.sqrt(x.a)
    return Dual(r, x.d / (2.0 * r))


def e001():
    """Young's modulus along [001]: 1/S11, S11 = (C11 + C12)/((C11 - C12)(C11 + 2 C12))."""
    return (C11 - C12) * (C11 + 2.0 * C12) / (C11 + C12)


def reduced_curve(theta, flow: Flow, rate, dt, T, rho0):
    """sigma33_t, t = 1..T, of the scalar recursion, as Duals in theta =
    (tau0, k1, k2, n) (the derivative directions are the unit vectors)."""
    tau0, k1, k2, n = (Dual(theta[k], np.eye(4)[k]) for k in range(4))
    E = e001()
    s6 = math.sqrt(6.0)
    p = Dual(0.0)
    rho = Dual(rho0)
    out = []
    for t in range(1, T + 1):
        E33 = -rate * dt * t
        tauc = tau0 + flow.alpha * flow.mu * flow.b * dsqrt(rho)

        def rate_mag(sig):           # gdot0 |sigma / (sqrt6 tauc)|^n, sigma < 0
            return flow.gdot0 * dexp(n * dlog((-1.0 * sig) / (s6 * tauc)))

        # Newton on f(sigma) = sigma/E + p - dt (8/sqrt6) g(sigma) - E33 (compression,
        # sigma < 0); started from the elastic trial stress, with halving to keep sigma < 0
        sig = Dual(min(E * (E33 - p.a), -1e-3))
        for _ in range(200):
            g = rate_mag(sig)
            f = sig / E + p - dt * 8.0 / s6 * g - E33
            fp = 1.0 / E + dt * 8.0 / s6 * n.a * g.a / (-sig.a)
            step = f.a / fp
            new = sig - f / fp
            while new.a >= 0.0:
                new = Dual(0.5 * sig.a, new.d)
            done = abs(step) <= 1e-15 * abs(sig.a)
            sig = new
            if done:
                break
        g = rate_mag(sig)
        # one more Newton pass so the derivative parts are consistent at the root
        f = sig / E + p - dt * 8.0 / s6 * g - E33
        fp = 1.0 / E + dt * 8.0 / s6 * n.a * g.a / (-sig.a)
        sig = sig - f / fp
        g = rate_mag(sig)
        p = p - dt * 8.0 / s6 * g
        rho = rho + dt * (k1 * dsqrt(rho) - k2 * rho) * 8.0 * g
        out.append(sig)
    return out


def cube_crystal(shape=(2, 2, 2), rho0=1e12):
    V = int(np.prod(shape))
    quat = np.repeat(np.array([1.0, 0, 0, 0])[:, None], V, axis=1)
    return quat, np.full(V, rho0)


RATE, DT = 1e-3, 2.0


def test_reduced_steady_state_closed_form():
    """k1 = k2 = 0: the recursion reaches |sigma33| = sqrt6 tauc
    (sqrt6 rate / (8 gdot0))^(1/n) within a few increments, with
    d sigma / d tau0 = sigma / tauc and d sigma / d n = -sigma ln(sqrt6 rate /
    (8 gdot0)) / n^2."""
    f = Flow(k1=0.0, k2=0.0)
    s = reduced_curve(f.theta(), f, RATE, DT, 12, 1e12)[-1]
    tauc = f.tau0 + f.alpha * f.mu * f.b * 1e6
    a = math.sqrt(6.0) * RATE / (8.0 * f.gdot0)
    want = -math.sqrt(6.0) * tauc * a ** (1.0 / f.n)
    assert abs(s.a - want) < 1e-13 * abs(want)
    assert abs(s.d[0] - want / tauc) < 1e-12 * abs(want / tauc)
    assert abs(s.d[3] - (-want * math.log(a) / f.n ** 2)) < 1e-12 * abs(want * math.log(a) / f.n ** 2)


@pytest.mark.parametrize("flow", [Flow(), Flow(k1=1.6e8, k2=4.0, n=7.5, tau0=8.0)])
def test_oracle_curve_equals_scalar_recursion(flow):
    """stress_curve of the field oracle equals the scalar recursion at every
    increment (fields uniform, lateral stresses free)."""
    quat, rho = cube_crystal()
    T = 6
    s, reps = stress_curve((2, 2, 2), quat, rho, flow, Loading(), T)
    red = reduced_curve(flow.theta(), flow, RATE, DT, T, 1e12)
    want = np.array([x.a for x in red])
    assert np.max(np.abs(s - want)) < 1e-11 * np.max(np.abs(want)), (s, want)
    assert all(r["converged"] for r in reps)


def _target(T):
    f = Flow()
    th = f.theta() * np.array([1.05, 0.95, 1.05, 0.95])
    return np.array([x.a for x in reduced_curve(th, f.with_theta(th), RATE, DT, T, 1e12)])


def _exact_gradient(flow, T, target):
    red = reduced_curve(flow.theta(), flow, RATE, DT, T, 1e12)
    g = np.zeros(4)
    for t, x in enumerate(red):
        g += 2.0 / T * (x.a - target[t]) * x.d
    return g


def test_fd_gradient_equals_exact_gradient():
    """fd_gradient of the oracle's curve loss = the exact gradient of the
    recursion, every component within 1e-6 relative (the components differ in
    magnitude and sign, so a swapped or mis-stepped component fails)."""
    f = Flow()
    T = 4
    tgt = _target(T)
    g_exact = _exact_gradient(f, T, tgt)
    quat, rho = cube_crystal()
    g_fd = fd_gradient((2, 2, 2), quat, rho, f, Loading(), T, tgt)
    assert np.all(np.abs(g_exact) > 0)
    assert np.max(np.abs(g_fd - g_exact) / np.abs(g_exact)) < 1e-6, (g_fd, g_exact)


def test_taylor_remainder_is_second_order():
    """L(theta + h v) - L(theta) - h g.v with the oracle's loss and the exact
    gradient shrinks 4x per halving of h (a wrong gradient leaves an O(h)
    remainder)."""
    f = Flow()
    T = 4
    tgt = _target(T)
    g = _exact_gradient(f, T, tgt)
    quat, rho = cube_crystal()
    th0 = f.theta()
    v = th0 * np.array([0.6, -0.8, 0.5, 0.3])

    def L(th):
        s, _ = stress_curve((2, 2, 2), quat, rho, f.with_theta(th), Loading(), T)
        return curve_loss(s, tgt)

    L0 = L(th0)
    rem = []
    for h in (4e-3, 2e-3, 1e-3):
        rem.append(abs(L(th0 + h * v) - L0 - h * g @ v))
    r1, r2 = rem[0] / rem[1], rem[1] / rem[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, rem
    # and the first-order term is what cancels: with g = 0 the remainder is O(h)
    assert abs(L(th0 + 1e-3 * v) - L0) > 20 * rem[2]


def test_halving_the_increment_is_first_order():
    """P13: a two-grain polycrystal compressed to 1 % strain with increments
    of 2e-3, 1e-3 and 5e-4: the end stress changes by O(increment), the
    second change about half the first."""
    shape = (4, 4, 2)
    V = 32
    rng = np.random.default_rng(11)
    q = synth.random_quaternions(2, rng)
    grains = (np.arange(V) % 4 >= 2).astype(int)
    quat = np.ascontiguousarray(q[grains].T)
    rho = np.full(V, 1e12)
    end = []
    for n_inc in (5, 10, 20):
        dt = 0.01 / RATE / n_inc
        o = Oracle(shape, quat, rho)
        for _ in range(n_inc):
            r = o.increment(Loading(dt=dt), tol=1e-11, max_iter=2000)
            assert r["converged"]
        end.append(r["Sigma"][2])
    d1, d2 = abs(end[0] - end[1]), abs(end[1] - end[2])
    assert d2 < d1 and 0.35 < d2 / d1 < 0.65, (end, d1, d2)
