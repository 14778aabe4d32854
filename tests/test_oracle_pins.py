"""Pins of the CPU oracle against values fixed independently of it.

Each test checks the oracle against something the mechanics or the paper
fixes (closed forms, bounds, identities, invariants, textbook special cases),
chosen so that a plausible slip anywhere (a wrong sign, a transposed operand,
a missing factor, a wrong axis) fails at least one of them.
"""
import numpy as np
import pytest
from scipy.optimize import root

import synth
from oracle import Oracle, Flow, Loading, default_c0, CU
from oracle import local as L
from oracle.crystal import slip_systems, voxel_material
from oracle.green import frequencies, gamma_mandel, gamma_field, green_apply
from oracle.tensors import (c4_to_mandel, cubic_c4, isotropic_c4, mandel_to_tensor,
                            mandel_to_voigt, quat_to_rot, rotate_c4, tensor_to_mandel,
                            voigt_to_mandel)

C11, C12, C44 = CU["C11"], CU["C12"], CU["C44"]
IDQ = np.array([1.0, 0.0, 0.0, 0.0])


def uniform(shape, q):
    V = int(np.prod(shape))
    return np.repeat(np.asarray(q, float)[:, None], V, axis=1), np.full(V, 1e12)


def q_axis_angle(axis, ang):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    return np.concatenate([[np.cos(ang / 2)], np.sin(ang / 2) * a])


def q_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def elastic_flow():
    return Flow(gdot0=0.0)


def voigt_c0(c11=C11, c12=C12, c44=C44):
    """Elastic reference medium for the purely elastic pins."""
    K = (c11 + 2 * c12) / 3
    mu = (c11 - c12 + 3 * c44) / 5
    return K - 2 * mu / 3, mu


# ---------------------------------------------------------------- tensors ---
def test_mandel_round_trip_and_contraction():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((3, 3)); A = A + A.T
    B = rng.standard_normal((3, 3)); B = B + B.T
    a, b = tensor_to_mandel(A), tensor_to_mandel(B)
    assert np.allclose(mandel_to_tensor(a), A)
    assert np.isclose(a @ b, np.sum(A * B))                      # a:b
    v = np.array([A[0, 0], A[1, 1], A[2, 2], A[1, 2], A[0, 2], A[0, 1]])
    assert np.allclose(voigt_to_mandel(v), a)


def test_quaternion_rotation_is_active_crystal_to_sample():
    R = quat_to_rot(q_axis_angle([0, 0, 1], np.pi / 2))
    assert np.allclose(R @ [1, 0, 0], [0, 1, 0])                  # x_c -> y_s
    rng = np.random.default_rng(1)
    q = synth.random_quaternions(50, rng).T
    R = quat_to_rot(q)
    assert np.allclose(np.einsum("mij,mkj->mik", R, R), np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(R), 1.0)


def test_cubic_moduli_closed_forms():
    """Directional Young's moduli of cubic Cu from the compliances."""
    s11 = (C11 + C12) / ((C11 - C12) * (C11 + 2 * C12))
    s12 = -C12 / ((C11 - C12) * (C11 + 2 * C12))
    s44 = 1.0 / C44
    E100 = 1 / s11
    E111 = 1 / (s11 - 2 * (s11 - s12 - s44 / 2) / 3)
    assert np.isclose(E100, 66688.75, rtol=1e-6)
    assert np.isclose(E111, 191149.69, rtol=1e-6)
    # oracle compliance for a crystal with [111] along z
    q = q_axis_angle(np.cross([1, 1, 1], [0, 0, 1]), np.arccos(1 / np.sqrt(3)))
    _, S, _ = voxel_material(q[:, None], C11, C12, C44)
    assert np.isclose(1 / S[0, 2, 2], E111, rtol=1e-12)
    _, S, _ = voxel_material(IDQ[:, None], C11, C12, C44)
    assert np.isclose(1 / S[0, 2, 2], E100, rtol=1e-12)


# ----------------------------------------------------------- slip systems ---
def test_slip_systems_geometry():
    n, d = slip_systems()
    assert n.shape == d.shape == (12, 3)
    assert np.allclose(np.linalg.norm(n, axis=1), 1) and np.allclose(np.linalg.norm(d, axis=1), 1)
    assert np.allclose(np.sum(n * d, axis=1), 0)
    # 4 distinct {111} planes, 6 distinct <110> lines
    assert len({tuple(np.round(np.abs(x) * np.sqrt(3)).astype(int)) for x in n}) == 1
    dirs = {tuple(np.round(x * np.sqrt(2)).astype(int)) for x in d}
    dirs |= {tuple(-np.array(t)) for t in dirs}
    assert len(dirs) == 12


def test_schmid_factors_for_001_loading():
    """Uniaxial stress along [001]: 8 systems at Schmid factor 1/sqrt6, 4 at 0."""
    _, _, m = voxel_material(IDQ[:, None], C11, C12, C44)
    sig = voigt_to_mandel(np.array([0, 0, 1.0, 0, 0, 0]))
    tau = L.resolved_shear(sig[None], m)[0]
    assert np.allclose(np.sort(np.abs(tau)), [0] * 4 + [1 / np.sqrt(6)] * 8, atol=1e-15)


def test_gdot_field_uniaxial_single_crystal():
    """Slip-rate field under uniaxial [001] stress on an unrotated crystal:
    system a carries gdot0 |s f_a / tauc|^n sign(s f_a) with the Schmid factor
    f_a = (n_a . e3)(d_a . e3) taken from the plane normals and directions
    (eight systems at |f| = 1/sqrt6, four at 0), in the order of the system
    list, and the rates sum to a compressive plastic rate along e3."""
    shape = (8, 8, 8)
    quat, rho = uniform(shape, IDQ)
    o = Oracle(shape, quat, rho)
    s = -80.0
    o.sigma = np.tile(voigt_to_mandel(np.array([0, 0, s, 0, 0, 0.0])), (o.nvox, 1))
    g = o.field("gdot")
    assert g.shape == (12, o.nvox)
    n, d = slip_systems()
    f = n[:, 2] * d[:, 2]
    tauc = 5.0 + 0.5 * 47337.0 * 2.56e-10 * 1e6
    want = 1e-3 * np.abs(s * f / tauc) ** 10 * np.sign(s * f)
    assert np.allclose(np.sort(np.abs(f)), [0] * 4 + [1 / np.sqrt(6)] * 8, atol=1e-15)
    assert np.allclose(g, want[:, None], rtol=1e-13, atol=0)
    # plastic rate along e3: sum_a gdot_a f_a < 0 under compression
    assert (want * f).sum() < 0


def test_plastic_rate_is_traceless():
    st = synth.random_voxel_states(64, seed=3)
    _, _, m = voxel_material(st["quat"], C11, C12, C44)
    sig = voigt_to_mandel(st["lam"]).T
    tauc = np.full(64, 10.0)
    ep = L.plastic_rate(sig, m, tauc, 1e-3, 10.0)
    assert np.abs(ep[:, :3].sum(axis=1)).max() < 1e-15 * np.abs(ep).max()


# ------------------------------------------------------------ local solve ---
@pytest.fixture(scope="module")
def local_case():
    st = synth.random_voxel_states(200, seed=4)
    _, S, m = voxel_material(st["quat"], C11, C12, C44)
    lam0, mu0 = default_c0(C11, C12, C44)
    C0inv = np.linalg.inv(c4_to_mandel(isotropic_c4(lam0, mu0)))
    tauc = 5.0 + 0.5 * 47337.0 * 2.56e-10 * np.sqrt(st["rho"])
    args = dict(lam=voigt_to_mandel(st["lam"]).T, e=voigt_to_mandel(st["e"]).T,
                epsp=voigt_to_mandel(st["epsp"]).T, tauc=tauc, S=S, m=m, C0inv=C0inv,
                gdot0=1e-3, n=10.0, dt=2.0)
    return args


def test_local_residual_vanishes(local_case):
    a = local_case
    sig, it, nfail = L.local_solve(a["lam"], a["e"], a["epsp"], a["tauc"], a["S"], a["m"],
                                   a["C0inv"], a["gdot0"], a["n"], a["dt"])
    assert nfail == 0
    r = L.residual(sig, a["lam"], a["e"], a["epsp"], a["S"], a["C0inv"], a["m"], a["tauc"],
                   a["gdot0"], a["n"], a["dt"])
    scale = np.abs(a["C0inv"]).max() * np.abs(sig).max()
    assert np.abs(r).max() < 1e-13 * scale


def test_local_jacobian_matches_finite_differences(local_case):
    a = local_case
    sig = a["lam"][:20] * 0.3
    args = (a["lam"][:20], a["e"][:20], a["epsp"][:20], a["S"][:20], a["C0inv"], a["m"][:20],
            a["tauc"][:20], a["gdot0"], a["n"], a["dt"])
    J = L.jacobian(sig, a["S"][:20], a["C0inv"], a["m"][:20], a["tauc"][:20], a["gdot0"], a["n"],
                   a["dt"])
    h = 1e-4
    for k in range(6):
        dp, dm = sig.copy(), sig.copy()
        dp[:, k] += h
        dm[:, k] -= h
        col = (L.residual(dp, *args) - L.residual(dm, *args)) / (2 * h)
        assert np.allclose(J[:, :, k], col, rtol=1e-6, atol=1e-12)
    # gradient of the potential is the residual
    for k in range(6):
        dp, dm = sig.copy(), sig.copy()
        dp[:, k] += h
        dm[:, k] -= h
        g = (L.potential(dp, *args) - L.potential(dm, *args)) / (2 * h)
        assert np.allclose(g, L.residual(sig, *args)[:, k], rtol=1e-6, atol=1e-12)


def test_local_solution_independent_of_start(local_case):
    a = local_case
    base = dict(lam=a["lam"], e=a["e"], epsp=a["epsp"], tauc=a["tauc"], S=a["S"], m=a["m"],
                C0inv=a["C0inv"], gdot0=a["gdot0"], n=a["n"], dt=a["dt"])
    s1, _, f1 = L.local_solve(**base)
    s2, _, f2 = L.local_solve(**base, sig0=np.zeros_like(a["lam"]))
    s3, _, f3 = L.local_solve(**base, sig0=-3 * a["lam"])
    assert f1 == f2 == f3 == 0
    assert np.abs(s1 - s2).max() < 1e-11 * np.abs(s1).max()
    assert np.abs(s1 - s3).max() < 1e-11 * np.abs(s1).max()


# --------------------------------------------------------- Green operator ---
def test_green_closed_form_and_identities():
    lam0, mu0 = 70000.0, 30000.0
    C0_4 = isotropic_c4(lam0, mu0)
    C0 = c4_to_mandel(C0_4)
    rng = np.random.default_rng(5)
    nv = rng.standard_normal((30, 3))
    nv /= np.linalg.norm(nv, axis=1, keepdims=True)
    G = gamma_mandel(nv, C0_4)
    for k in range(30):
        n = nv[k]
        # closed form for an isotropic medium (Moulinec-Suquet), Mandel
        Gt = np.zeros((3, 3, 3, 3))
        d = np.eye(3)
        for i in range(3):
            for j in range(3):
                for p in range(3):
                    for q in range(3):
                        Gt[i, j, p, q] = ((d[p, i] * n[q] * n[j] + d[q, i] * n[p] * n[j]
                                           + d[p, j] * n[q] * n[i] + d[q, j] * n[p] * n[i]) / (4 * mu0)
                                          - (lam0 + mu0) / (mu0 * (lam0 + 2 * mu0))
                                          * n[i] * n[j] * n[p] * n[q])
        assert np.allclose(G[k], c4_to_mandel(Gt), rtol=1e-13, atol=1e-19)
        assert np.allclose(G[k] @ C0 @ G[k], G[k], atol=1e-18)          # projector
        a = rng.standard_normal(3)
        s = tensor_to_mandel(0.5 * (np.outer(n, a) + np.outer(a, n)))
        assert np.allclose(G[k] @ C0 @ s, s, atol=1e-13)                  # compatible fields
        tau = rng.standard_normal(6)
        sig = tau - C0 @ (G[k] @ tau)                                     # equilibrated
        assert np.abs(mandel_to_tensor(sig) @ n).max() < 1e-10 * np.abs(tau).max()


def test_spectral_update_of_one_cosine_mode():
    """tau = t0 cos(2 pi k.x / N) must give e = E - Gamma0(n) t0 cos(...)."""
    shape = (8, 16, 4)
    n0, n1, n2 = shape
    q, rho = uniform(shape, IDQ)
    o = Oracle(shape, q, rho)
    rng = np.random.default_rng(6)
    t0 = rng.standard_normal(6)
    E = rng.standard_normal(6) * 1e-3
    z, y, x = np.meshgrid(np.arange(n2), np.arange(n1), np.arange(n0), indexing="ij")
    for k in [(1, 0, 0), (0, 3, 0), (2, -5, 1), (3, 1, -1)]:
        ph = 2 * np.pi * (k[0] * x / n0 + k[1] * y / n1 + k[2] * z / n2)
        tau = (t0[:, None] * np.cos(ph).reshape(1, -1)).T
        e = o.spectral_update(tau, E)
        xi = np.array([k[0] / n0, k[1] / n1, k[2] / n2])
        G = gamma_mandel((xi / np.linalg.norm(xi))[None], o.C0_4)[0]
        want = E[None, :] - (G @ t0)[None, :] * np.cos(ph).reshape(-1, 1)
        assert np.abs(e - want).max() < 1e-13 * np.abs(G @ t0).max()


def test_nyquist_mode_is_filtered_to_zero_stress():
    shape = (8, 8, 8)
    q, rho = uniform(shape, IDQ)
    o = Oracle(shape, q, rho)
    t0 = np.array([1.0, -2.0, 0.5, 0.3, -0.2, 0.7])
    x = np.tile(np.arange(8), 64)
    tau = (t0[:, None] * ((-1.0) ** x)[None]).T
    e = o.spectral_update(tau, np.zeros(6))
    assert np.allclose(e, -(tau @ o.C0inv.T), atol=1e-15)


def test_fft_convention_against_brute_force_dft():
    rng = np.random.default_rng(7)
    f = rng.standard_normal((4, 4, 4))
    F = np.zeros((4, 4, 4), complex)
    for a in range(4):
        for b in range(4):
            for c in range(4):
                for z in range(4):
                    for y in range(4):
                        for x in range(4):
                            F[a, b, c] += f[z, y, x] * np.exp(-2j * np.pi * (a * z + b * y + c * x) / 4)
    assert np.allclose(np.fft.fftn(f), F, atol=1e-12)
    kx, ky, kz = frequencies((4, 4, 4))
    assert list(kx) == [0, 1, -2, -1]


# -------------------------------------------------------- whole-path pins ---
def test_single_crystal_elastic_moduli_and_uniform_fields():
    shape = (8, 8, 8)
    for q, Ewant in [(IDQ, 66688.75),
                     (q_axis_angle(np.cross([1, 1, 1], [0, 0, 1]), np.arccos(1 / np.sqrt(3))),
                      191149.69)]:
        qq, rho = uniform(shape, q)
        o = Oracle(shape, qq, rho, flow=elastic_flow(), c0=voigt_c0())
        r = o.increment(Loading(), tol=1e-13, max_iter=500)
        assert r["converged"]
        assert np.isclose(r["Sigma"][2] / r["E"][2], Ewant, rtol=1e-6)
        s = o.field("sigma")
        assert np.abs(s - s.mean(axis=1, keepdims=True)).max() < 1e-12 * np.abs(s).max()


def test_single_crystal_viscoplastic_steady_state():
    """[001] crystal, no hardening: |s33| -> sqrt6 tauc (sqrt6 |Edot| / (8 gdot0))^(1/n)."""
    shape = (8, 8, 8)
    qq, rho = uniform(shape, IDQ)
    f = Flow(k1=0.0, k2=0.0)
    o = Oracle(shape, qq, rho, flow=f)
    for _ in range(12):
        r = o.increment(Loading(), tol=1e-13, max_iter=500)
    tauc = o.tauc()[0]
    want = np.sqrt(6) * tauc * (np.sqrt(6) * 1e-3 / (8 * f.gdot0)) ** (1 / f.n)
    assert np.isclose(-r["Sigma"][2], want, rtol=1e-10)
    assert np.isclose(want / tauc, 2.17608, rtol=1e-5)


def test_kocks_mecking_saturation_and_closed_form():
    """Single crystal: sqrt(rho) follows k1/k2 - (k1/k2 - sqrt rho0) exp(-k2 G / 2)."""
    shape = (8, 8, 8)
    qq, rho = uniform(shape, IDQ)
    f = Flow(k1=8e7, k2=10.0)
    o = Oracle(shape, qq, rho, flow=f)
    G = 0.0
    d = Loading()
    errs = []
    for _ in range(30):
        sig_prev_rho = o.rho[0]
        r = o.increment(d, tol=1e-12, max_iter=500)
        _, gdot = L.slip_rates(o.sigma[:1], o.m[:1], o.tauc(np.array([sig_prev_rho])), f.gdot0, f.n)
        G += d.dt * np.abs(gdot).sum()
        exact = (f.k1 / f.k2 - (f.k1 / f.k2 - 1e6) * np.exp(-f.k2 * G / 2)) ** 2
        errs.append(abs(o.rho[0] - exact) / exact)
    # explicit Euler in G: first-order error, small for these increments
    assert max(errs) < 0.05
    o2 = Oracle(shape, qq, np.full(512, (f.k1 / f.k2) ** 2), flow=f)
    o2.increment(d, tol=1e-12)
    assert np.allclose(o2.rho, (f.k1 / f.k2) ** 2, rtol=1e-14)             # fixed point


def test_hydrostatic_polycrystal():
    shape = (8, 8, 8)
    w = synth.Workload("p", shape, 5, "uniform", 1, 1e-6, seed=9)
    q, rho, _ = synth.make_microstructure(w)
    o = Oracle(shape, q, rho, flow=elastic_flow(), c0=voigt_c0())
    load = Loading(Edot=np.array([1e-3, 1e-3, 1e-3, 0, 0, 0]), strain_ctrl=np.ones(6, int))
    o.increment(load, tol=1e-13, max_iter=200)
    K = (C11 + 2 * C12) / 3
    s = o.field("sigma")
    want = np.array([3 * K * 2e-3] * 3 + [0] * 3)
    assert np.abs(s - want[:, None]).max() < 1e-10 * 3 * K * 2e-3


def test_isotropic_limit_polycrystal():
    shape = (8, 8, 8)
    c11, c12 = 200000.0, 100000.0
    c44 = (c11 - c12) / 2
    w = synth.Workload("p", shape, 6, "uniform", 1, 1e-6, seed=10)
    q, rho, _ = synth.make_microstructure(w)
    o = Oracle(shape, q, rho, C11=c11, C12=c12, C44=c44, flow=elastic_flow(),
               c0=voigt_c0(c11, c12, c44))
    r = o.increment(Loading(), tol=1e-13, max_iter=300)
    K, mu = (c11 + 2 * c12) / 3, c44
    assert np.isclose(r["Sigma"][2] / r["E"][2], 9 * K * mu / (3 * K + mu), rtol=1e-10)
    s = o.field("sigma")
    assert np.abs(s - s.mean(axis=1, keepdims=True)).max() < 1e-9 * np.abs(s).max()


def _laminate(axis, plastic):
    """Two-grain laminate normal to ``axis``: exact piecewise-uniform solution."""
    N = 8
    shape = (N, N, N)
    qa = q_axis_angle([1, 2, 3], 0.7)
    qb = q_axis_angle([-2, 1, 0.5], 1.9)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    coord = [x, y, z][axis].reshape(-1)
    inA = coord < N // 2
    quat = np.where(inA[None], qa[:, None], qb[:, None])
    rho = np.full(N ** 3, 1e12)
    flow = Flow() if plastic else elastic_flow()
    o = Oracle(shape, quat, rho, flow=flow, c0=None if plastic else voigt_c0())
    _, SA, mA = voxel_material(qa[:, None], C11, C12, C44)
    _, SB, mB = voxel_material(qb[:, None], C11, C12, C44)
    load = Loading()
    # tangential strain / normal traction components (tensor index pairs)
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    tang = [k for k, (i, j) in enumerate(pairs) if i != axis and j != axis]
    norm = [k for k, (i, j) in enumerate(pairs) if i == axis or j == axis]
    E33 = 0.0
    epA = np.zeros(6); epB = np.zeros(6)
    rA = rB = 1e12
    for inc in range(3 if plastic else 1):
        E33 += -2e-3
        tcA = flow.tau0 + flow.alpha * flow.mu * flow.b * np.sqrt(rA)
        tcB = flow.tau0 + flow.alpha * flow.mu * flow.b * np.sqrt(rB)

        def strain(s, S, m, ep, tc, n):
            return S[0] @ s + ep + load.dt * L.plastic_rate(s[None], m, np.array([tc]), flow.gdot0, n)[0]

        def eqs(u, n=flow.n):
            sA, sB, Es = u[:6] * 1e2, u[6:12] * 1e2, u[12:]
            eA = strain(sA, SA, mA, epA, tcA, n)
            eB = strain(sB, SB, mB, epB, tcB, n)
            E = np.array([Es[0], Es[1], E33, Es[2], Es[3], Es[4]])
            res = [(eA - eB)[tang] * 1e3, (sA - sB)[norm] * 1e-2,
                   (0.5 * (eA + eB) - E) * 1e3, (0.5 * (sA + sB))[[0, 1, 3, 4, 5]] * 1e-2]
            return np.concatenate(res)

        # continuation in the rate exponent from a linear viscous law
        u = np.zeros(17)
        for n in (list(np.linspace(1.0, flow.n, 19)) if plastic else [flow.n]):
            u = root(eqs, u, args=(n,), method="hybr", tol=1e-15).x
        assert np.abs(eqs(u)).max() < 1e-11
        sA, sB = u[:6] * 1e2, u[6:12] * 1e2
        r = o.increment(load, tol=1e-13, max_iter=3000)
        assert r["converged"]
        s = o.sigma
        scale = np.abs(sA).max()
        assert np.abs(s[inA] - sA).max() < 1e-8 * scale, (axis, inc)
        assert np.abs(s[~inA] - sB).max() < 1e-8 * scale, (axis, inc)
        # state update of the exact solution
        _, gA = L.slip_rates(sA[None], mA, np.array([tcA]), flow.gdot0, flow.n)
        _, gB = L.slip_rates(sB[None], mB, np.array([tcB]), flow.gdot0, flow.n)
        epA = epA + load.dt * (gA @ mA[0])[0]
        epB = epB + load.dt * (gB @ mB[0])[0]
        rA = rA + load.dt * (flow.k1 * np.sqrt(rA) - flow.k2 * rA) * np.abs(gA).sum()
        rB = rB + load.dt * (flow.k1 * np.sqrt(rB) - flow.k2 * rB) * np.abs(gB).sum()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_laminate_elastic(axis):
    _laminate(axis, plastic=False)


def test_laminate_viscoplastic():
    _laminate(2, plastic=True)


@pytest.fixture(scope="module")
def poly8():
    shape = (8, 8, 8)
    w = synth.Workload("p", shape, 6, "lognormal", 2, 1e-6, seed=13)
    q, rho, _ = synth.make_microstructure(w)
    return shape, q.reshape(4, -1), rho.reshape(-1)


def test_voigt_reuss_bounds(poly8):
    shape, q, rho = poly8
    o = Oracle(shape, q, rho, flow=elastic_flow(), c0=voigt_c0())
    r = o.increment(Loading(), tol=1e-12, max_iter=500)
    Eeff = r["Sigma"][2] / r["E"][2]
    Cm = o.C.mean(axis=0)
    Sm = o.S.mean(axis=0)
    E_voigt = 1 / np.linalg.inv(Cm)[2, 2]
    E_reuss = 1 / Sm[2, 2]
    assert E_reuss < Eeff < E_voigt


def test_mean_strain_hill_mandel_and_bc(poly8):
    shape, q, rho = poly8
    o = Oracle(shape, q, rho)
    for _ in range(2):
        r = o.increment(Loading(), tol=1e-11, max_iter=3000)
    e = voigt_to_mandel(o.field("strain"))
    s = voigt_to_mandel(o.field("sigma"))
    assert np.allclose(e.mean(axis=1), voigt_to_mandel(r["E"]), atol=1e-15)
    assert np.isclose(r["E"][2], -4e-3, rtol=1e-14)
    S = s.mean(axis=1)
    assert np.abs(S[[0, 1, 3, 4, 5]]).max() < 1e-9 * abs(S[2])
    hm = np.mean(np.sum(s * e, axis=0))
    assert abs(hm - S @ e.mean(axis=1)) < 1e-9 * abs(hm)
    # equilibrium: divergence-free stress in Fourier space
    sh = np.fft.fftn(s.reshape(6, 8, 8, 8), axes=(1, 2, 3))
    kx, ky, kz = frequencies(shape)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    nyq = (np.abs(KX) == 4) | (np.abs(KY) == 4) | (np.abs(KZ) == 4)
    T = mandel_to_tensor(np.moveaxis(sh, 0, -1))
    div = np.einsum("zyxij,zyxj->zyxi", T, np.stack([KX, KY, KZ], -1))
    assert np.abs(div[~nyq]).max() < 1e-8 * np.abs(sh[:, 0, 0, 0]).max()
    assert np.abs(sh[:, nyq]).max() < 1e-8 * np.abs(sh[:, 0, 0, 0]).max()


def test_shift_and_cubic_symmetry_invariance(poly8):
    shape, q, rho = poly8
    o1 = Oracle(shape, q, rho)
    r1 = o1.increment(Loading(), tol=1e-12, max_iter=3000)
    # circular shift of the microstructure by (3, 1, 5) voxels
    sh = lambda a: np.roll(a.reshape(a.shape[0], 8, 8, 8), (5, 1, 3), axis=(1, 2, 3)).reshape(a.shape[0], -1)
    o2 = Oracle(shape, sh(q), sh(rho[None])[0])
    r2 = o2.increment(Loading(), tol=1e-12, max_iter=3000)
    assert np.allclose(r2["Sigma"], r1["Sigma"], rtol=1e-9, atol=1e-9)
    assert np.allclose(o2.field("sigma"), sh(o1.field("sigma")), atol=1e-8)
    # a cubic symmetry operation of the crystal leaves everything unchanged
    s4 = q_axis_angle([0, 0, 1], np.pi / 2)
    q3 = np.stack([q_mul(q[:, i], s4) for i in range(q.shape[1])], axis=1)
    o3 = Oracle(shape, q3, rho)
    r3 = o3.increment(Loading(), tol=1e-12, max_iter=3000)
    assert np.allclose(r3["Sigma"], r1["Sigma"], rtol=1e-9, atol=1e-9)
    assert np.allclose(o3.field("sigma"), o1.field("sigma"), atol=1e-8)


def test_reference_medium_does_not_change_the_fixed_point(poly8):
    shape, q, rho = poly8
    out = []
    K = (C11 + 2 * C12) / 3
    for mu0 in (2000.0, 8000.0):
        o = Oracle(shape, q, rho, c0=(K - 2 * mu0 / 3, mu0))
        r = o.increment(Loading(), tol=1e-12, max_iter=5000)
        assert r["converged"]
        out.append(o.field("sigma"))
    assert np.abs(out[0] - out[1]).max() < 1e-8 * np.abs(out[0]).max()


def test_global_quarter_turn_about_z_permutes_the_fields():
    """P11: turning the whole polycrystal by 90 degrees about z (orientations
    q -> r q, voxel (x, y) -> (n-1-y, x)) under compression along z with free
    lateral faces (a loading the turn leaves unchanged) turns every field:
    s'11 = s22, s'22 = s11, s'33 = s33, s'23 = s13, s'13 = -s23, s'12 = -s12
    at the turned voxel."""
    shape = (8, 8, 4)
    g = [np.random.default_rng(s) for s in np.random.SeedSequence(31).spawn(4)]
    grains = synth.voronoi_grains(shape, 4, g[0])
    q = synth.random_quaternions(4, g[1])
    quat = np.moveaxis(q[grains], -1, 0)                    # (4, z, y, x)
    rho = synth.lognormal_rho(shape, 1e12, 0.3, g[2])       # (z, y, x)

    def turn(f):          # field [..., z, y, x] -> turned grid
        return np.flip(np.swapaxes(f, -1, -2), axis=-1)

    r = q_axis_angle([0, 0, 1], np.pi / 2)
    quat2 = turn(np.einsum("ij,j...->i...", np.array([q_mul(r, e) for e in np.eye(4)]).T, quat))
    quat2 = np.where(quat2[0:1] < 0, -quat2, quat2)
    o1 = Oracle(shape, quat.reshape(4, -1), rho.reshape(-1))
    o2 = Oracle(shape, quat2.reshape(4, -1), turn(rho).reshape(-1))
    for _ in range(2):
        r1 = o1.increment(Loading(), tol=1e-12, max_iter=3000)
        r2 = o2.increment(Loading(), tol=1e-12, max_iter=3000)
    s1 = o1.field("sigma").reshape(6, 4, 8, 8)
    s2 = o2.field("sigma").reshape(6, 4, 8, 8)
    want = np.stack([s1[1], s1[0], s1[2], s1[4], -s1[3], -s1[5]])
    scale = np.abs(s1).max()
    assert np.abs(s2 - turn(want)).max() < 1e-9 * scale
    e1 = o1.field("epsp").reshape(6, 4, 8, 8)
    e2 = o2.field("epsp").reshape(6, 4, 8, 8)
    wante = np.stack([e1[1], e1[0], e1[2], e1[4], -e1[3], -e1[5]])
    assert np.abs(e2 - turn(wante)).max() < 1e-9 * np.abs(e1).max()
    assert abs(r1["Sigma"][2] - r2["Sigma"][2]) < 1e-10 * abs(r1["Sigma"][2])
