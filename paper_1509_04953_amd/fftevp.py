"""Python binding of ``libfftevp.so`` (ctypes).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels. PyTorch supplies device memory (tensors whose ``data_ptr`` is handed
to the library) and the stream (``torch.cuda.current_stream()``). There is no
CPU fallback: if the library or a GPU is missing, construction raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "libfftevp.so"
_lib = None

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENONFINITE, ELOCAL, ESTATE = 0, 1, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
FIELDS = {"sigma": 0, "strain": 1, "epsp": 2, "rho": 3, "sigma_iter": 4, "strain_iter": 5, "gdot": 6,
          "rho_gnds": 7, "rho_gndet": 8, "rho_ssd": 9, "kappa": 10, "grain": 11, "quat": 12}
NPROF = 8
PROF_NAMES = ("local", "rotate", "yfwd", "zgamma", "yinv", "state", "adjoint", "gnd")
NCOMP = {"sigma": 6, "strain": 6, "epsp": 6, "rho": 1, "sigma_iter": 6, "strain_iter": 6, "gdot": 12,
         "rho_gnds": 12, "rho_gndet": 12, "rho_ssd": 12, "kappa": 1, "grain": 1, "quat": 4}


class Cubic(C.Structure):
    _fields_ = [("C11", C.c_double), ("C12", C.c_double), ("C44", C.c_double)]


class MRC(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("T", "Q_slip", "Q_bulk", "c1", "c2", "c3", "c4", "c5", "c6",
                                          "c7", "c8", "nu_D", "poisson")]


class DrxC(C.Structure):
    _fields_ = [("kc", C.c_double), ("q", C.c_double), ("s_nucl", C.c_double), ("s_soften", C.c_double)]


class GrowC(C.Structure):
    _fields_ = [("zeta", C.c_double), ("omega_gb", C.c_double), ("dx", C.c_double)]


class FlowC(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("tau0", "k1", "k2", "n", "gdot0", "alpha", "mu", "b")]


class LoadingC(C.Structure):
    _fields_ = [("Edot", C.c_double * 6), ("Sigma", C.c_double * 6),
                ("strain_ctrl", C.c_int * 6), ("dt", C.c_double)]


class OptsC(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("newton_max", C.c_int),
                ("c0_lambda", C.c_double), ("c0_mu", C.c_double)]


class ReportC(C.Structure):
    _fields_ = [("iters", C.c_int), ("newton_max_seen", C.c_int), ("newton_failed", C.c_int),
                ("err_c", C.c_double), ("err_bc", C.c_double), ("Sigma", C.c_double * 6),
                ("E", C.c_double * 6), ("rho_mean", C.c_double),
                ("newton_mean", C.c_double), ("linesearch_mean", C.c_double), ("l_eff", C.c_double)]


def library():
    """Load ``libfftevp.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is missing: run `python -m paper_1509_04953_amd.build`")
    lib = C.CDLL(str(_LIB_PATH))
    P, I, D, S = C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_size_t
    sig = {
        "fftevp_create": (I, [I, I, I, I, P, C.POINTER(P)]),
        "fftevp_destroy": (I, [P]),
        "fftevp_set_material": (I, [P, C.POINTER(Cubic), C.POINTER(FlowC)]),
        "fftevp_set_microstructure": (I, [P, P, P]),
        "fftevp_set_loading": (I, [P, C.POINTER(LoadingC)]),
        "fftevp_set_gnd": (I, [P, P, C.c_double, C.c_double]),
        "fftevp_set_law": (I, [P, I, C.POINTER(MRC)]),
        "fftevp_set_drx": (I, [P, C.POINTER(DrxC), P]),
        "fftevp_set_rotation": (I, [P, I]),
        "fftevp_drx_nucleate": (I, [P, P, C.POINTER(C.c_longlong)]),
        "fftevp_step": (I, [P, C.POINTER(OptsC), C.POINTER(ReportC)]),
        "fftevp_step_noalloc": (I, [P, C.POINTER(OptsC), C.POINTER(ReportC)]),
        "fftevp_redistribute": (I, [P, P, C.POINTER(OptsC), C.POINTER(ReportC)]),
        "fftevp_get_field": (I, [P, I, P]),
        "fftevp_state_bytes": (S, [P]),
        "fftevp_save_state": (I, [P, P]),
        "fftevp_load_state": (I, [P, P]),
        "fftevp_adjoint_bytes": (S, [P]),
        "fftevp_adjoint_increment": (I, [P, C.POINTER(OptsC), P, P, D, P, D]),
        "fftevp_set_profiling": (I, [P, I]),
        "fftevp_get_profile": (I, [P, D, C.POINTER(C.c_longlong), I]),
        "fftevp_status_string": (C.c_char_p, [I]),
        "fftevp_last_error": (C.c_char_p, [P]),
        "fftevp_pf_create": (I, [I, I, I, I, C.c_double, I, P, C.POINTER(P)]),
        "fftevp_pf_destroy": (I, [P]),
        "fftevp_pf_refine": (I, [P, P, P]),
        "fftevp_pf_import": (I, [P, P, P, I, P]),
        "fftevp_pf_steps": (I, [P, I]),
        "fftevp_pf_export": (I, [P, P, P]),
        "fftevp_pf_grains": (I, [P, P, P]),
        "fftevp_pf_last_error": (C.c_char_p, [P]),
        "fftevp_pf_dims": (I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(I)]),
        "fftevp_pf_step_count": (I, [C.c_double, C.c_double, C.c_double]),
        "fftevp_drx_grow": (I, [P, P, C.POINTER(GrowC), I, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class FftevpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fftevp status {status}: {msg}")
        self.status = status


@dataclass
class MaRoters:
    """Constants of the paper's dislocation-based law (Table 1; T, nu_D and
    the Poisson ratio as documented in include/fftevp.h)."""
    T: float = 473.0
    Q_slip: float = 3.3e-19
    Q_bulk: float = 3.51e-19
    c1: float = 0.5
    c2: float = 3.0
    c3: float = 3.0
    c4: float = 8.0e7
    c5: float = 10.0
    c6: float = 3.0e10
    c7: float = 7.0e-28
    c8: float = 0.24
    nu_D: float = 1.0e13
    poisson: float = 0.34


@dataclass
class Material:
    C11: float = 168400.0
    C12: float = 121400.0
    C44: float = 75400.0
    tau0: float = 5.0
    k1: float = 8.0e7
    k2: float = 10.0
    n: float = 10.0
    gdot0: float = 1.0e-3
    alpha: float = 0.5
    mu: float = 47337.0
    b: float = 2.56e-10

    def theta(self):
        return np.array([self.tau0, self.k1, self.k2, self.n])


@dataclass
class Load:
    Edot: tuple = (0.0, 0.0, -1.0e-3, 0.0, 0.0, 0.0)
    Sigma: tuple = (0.0,) * 6
    strain_ctrl: tuple = (0, 0, 1, 0, 0, 0)
    dt: float = 2.0


@dataclass
class Opts:
    tol: float = 1e-6
    max_iter: int = 1000
    newton_max: int = 50
    c0_lambda: float = 0.0
    c0_mu: float = 0.0


@dataclass
class Report:
    status: int
    iters: int
    newton_max_seen: int
    newton_failed: int
    err_c: float
    err_bc: float
    Sigma: np.ndarray
    E: np.ndarray
    rho_mean: float
    newton_mean: float = 0.0
    linesearch_mean: float = 0.0
    l_eff: float = 0.0


def _opts(o: Opts | None):
    o = o or Opts()
    return OptsC(o.tol, o.max_iter, o.newton_max, o.c0_lambda, o.c0_mu)


class Solver:
    """One FFT-EVP context on the current CUDA (HIP) device and stream."""

    def __init__(self, shape, precision: str = "fp64", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fftevp needs a GPU; no CPU fallback exists")
        self.torch = torch
        self.lib = library()
        self.shape = tuple(int(s) for s in shape)
        self.nvox = int(np.prod(self.shape))
        self.precision = precision
        prec = {"fp64": FP64, "mixed": MIXED}[precision]
        self.stream = stream or torch.cuda.current_stream()
        h = C.c_void_p()
        st = self.lib.fftevp_create(*self.shape, prec, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise FftevpError(st, self.lib.fftevp_status_string(st).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.fftevp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise FftevpError(st, self.lib.fftevp_last_error(self.h).decode())
        return st

    def set_material(self, m: Material):
        self._check(self.lib.fftevp_set_material(self.h, C.byref(Cubic(m.C11, m.C12, m.C44)),
                                                 C.byref(FlowC(m.tau0, m.k1, m.k2, m.n, m.gdot0,
                                                               m.alpha, m.mu, m.b))))
        self.material = m

    def _dev(self, a, shape):
        t = self.torch.as_tensor(a, dtype=self.torch.float64, device="cuda").reshape(shape).contiguous()
        return t

    def set_microstructure(self, quat, rho):
        q = self._dev(quat, (4, self.nvox))
        r = self._dev(rho, (self.nvox,))
        self._check(self.lib.fftevp_set_microstructure(self.h, C.c_void_p(q.data_ptr()),
                                                       C.c_void_p(r.data_ptr())))

    def set_law(self, law: "MaRoters | None"):
        """None: the power law; a MaRoters instance: the paper's law."""
        if law is None:
            self._check(self.lib.fftevp_set_law(self.h, 0, None))
            return
        c = MRC(*(getattr(law, k) for k, _ in MRC._fields_))
        self._check(self.lib.fftevp_set_law(self.h, 1, C.byref(c)))

    def set_drx(self, u, kc: float = 300e12, q: float = 4.4, s_nucl: float = 0.05, s_soften: float = 0.9):
        """DRX nucleation strengths from uniforms ``u`` (one per voxel, [0, 1))."""
        t = self._dev(u, (self.nvox,))
        self._check(self.lib.fftevp_set_drx(self.h, C.byref(DrxC(kc, q, s_nucl, s_soften)),
                                            C.c_void_p(t.data_ptr())))

    def drx_nucleate(self, u) -> int:
        """One nucleation test; ``u``: fresh uniforms for the redraws."""
        t = self._dev(u, (self.nvox,))
        n = C.c_longlong(0)
        self._check(self.lib.fftevp_drx_nucleate(self.h, C.c_void_p(t.data_ptr()), C.byref(n)))
        return int(n.value)

    def drx_grow(self, pf: "PhaseField", nsteps: int, zeta: float = 0.25, omega_gb: float = 0.625,
                 dx: float = 10.7e-6):
        """Grain growth on ``pf`` after nucleation; returns (voxels whose grain
        changed, of those now recrystallised)."""
        a, b = C.c_longlong(0), C.c_longlong(0)
        self._check(self.lib.fftevp_drx_grow(self.h, pf.h, C.byref(GrowC(zeta, omega_gb, dx)), int(nsteps),
                                             C.byref(a), C.byref(b)))
        return int(a.value), int(b.value)

    def set_rotation(self, on: bool = True):
        """Turn the lattice by its spin after every increment (include/fftevp.h)."""
        self._check(self.lib.fftevp_set_rotation(self.h, int(bool(on))))

    def drx_cycle(self, pf: "PhaseField", u, pf_steps: int, opts: Opts | None = None, zeta: float = 0.25,
                  omega_gb: float = 0.625, dx: float = 10.7e-6, redistribute: bool = True):
        """One increment of the coupled loop (Sec. 2.5): the mechanical solve,
        the nucleation test with fresh uniforms ``u``, ``pf_steps`` steps of
        grain growth, then the stress redistribution (the increment's solve
        repeated with the updated microstructure). Returns (report, nuclei,
        changed, recrystallised, redistribution report or None)."""
        before = self.save_state()
        r = self.step(opts, allow=(OK,))
        n = self.drx_nucleate(u)
        changed, rex = self.drx_grow(pf, pf_steps, zeta, omega_gb, dx)
        rr = self.redistribute(before, opts, allow=(OK,)) if redistribute else None
        return r, n, changed, rex, rr

    def redistribute(self, before, opts: Opts | None = None, allow=(OK, NOT_CONVERGED, ELOCAL)) -> Report:
        """fftevp_redistribute: the last increment's solve repeated from the
        snapshot ``before`` (taken just before it) with the current
        microstructure (stress redistribution after DRX, Sec. 2.5)."""
        r = ReportC()
        st = self._check(self.lib.fftevp_redistribute(self.h, C.c_void_p(before.data_ptr()),
                                                      C.byref(_opts(opts)), C.byref(r)), allow)
        return Report(st, r.iters, r.newton_max_seen, r.newton_failed, r.err_c, r.err_bc,
                      np.array(r.Sigma[:]), np.array(r.E[:]), r.rho_mean, r.newton_mean,
                      r.linesearch_mean, r.l_eff)

    def set_gnd(self, grains, l0: float = 21.4e-6, xi: float = 200.0):
        """Track GND densities (screw and edge, per slip system) from every
        committed increment on; ``grains`` holds one integer grain id per
        voxel, ``l0`` the grid spacing (m), ``xi`` the effective-length
        constant."""
        g = self.torch.as_tensor(np.asarray(grains).reshape(-1), dtype=self.torch.int32,
                                 device="cuda").contiguous()
        if g.numel() != self.nvox:
            raise ValueError("one grain id per voxel")
        self._check(self.lib.fftevp_set_gnd(self.h, C.c_void_p(g.data_ptr()), float(l0), float(xi)))

    def set_loading(self, ld: Load):
        c = LoadingC((C.c_double * 6)(*ld.Edot), (C.c_double * 6)(*ld.Sigma),
                     (C.c_int * 6)(*ld.strain_ctrl), ld.dt)
        self._check(self.lib.fftevp_set_loading(self.h, C.byref(c)))

    def step(self, opts: Opts | None = None, allow=(OK, NOT_CONVERGED, ELOCAL)) -> Report:
        r = ReportC()
        st = self._check(self.lib.fftevp_step(self.h, C.byref(_opts(opts)), C.byref(r)), allow)
        return Report(st, r.iters, r.newton_max_seen, r.newton_failed, r.err_c, r.err_bc,
                      np.array(r.Sigma[:]), np.array(r.E[:]), r.rho_mean, r.newton_mean,
                      r.linesearch_mean, r.l_eff)

    def step_noalloc(self, opts: Opts | None = None, allow=(OK, NOT_CONVERGED, ELOCAL)) -> Report:
        """fftevp_step_noalloc: the same increment with its scratch in the
        library's static device array (no allocation in the call)."""
        r = ReportC()
        st = self._check(self.lib.fftevp_step_noalloc(self.h, C.byref(_opts(opts)), C.byref(r)), allow)
        return Report(st, r.iters, r.newton_max_seen, r.newton_failed, r.err_c, r.err_bc,
                      np.array(r.Sigma[:]), np.array(r.E[:]), r.rho_mean, r.newton_mean,
                      r.linesearch_mean, r.l_eff)

    def field(self, name: str):
        n = NCOMP[name]
        out = self.torch.empty((n, self.nvox) if n > 1 else (self.nvox,), dtype=self.torch.float64,
                               device="cuda")
        self._check(self.lib.fftevp_get_field(self.h, FIELDS[name], C.c_void_p(out.data_ptr())))
        return out

    def state_bytes(self) -> int:
        return int(self.lib.fftevp_state_bytes(self.h))

    def save_state(self, out=None):
        if out is None:
            out = self.torch.empty(self.state_bytes(), dtype=self.torch.uint8, device="cuda")
        self._check(self.lib.fftevp_save_state(self.h, C.c_void_p(out.data_ptr())))
        return out

    def load_state(self, buf):
        self._check(self.lib.fftevp_load_state(self.h, C.c_void_p(buf.data_ptr())))

    def set_profiling(self, on, classes=None):
        """Time kernel classes with HIP events: all when ``classes`` is None,
        else the given names from PROF_NAMES."""
        mask = 0
        if on:
            names = PROF_NAMES if classes is None else classes
            for n in names:
                mask |= 1 << PROF_NAMES.index(n)
        self._check(self.lib.fftevp_set_profiling(self.h, mask))

    def profile(self, reset=True):
        """Per kernel class: (summed ms, launches) from HIP events."""
        ms = (C.c_double * NPROF)()
        n = (C.c_longlong * NPROF)()
        self._check(self.lib.fftevp_get_profile(self.h, ms, n, int(reset)))
        return {name: (ms[k], n[k]) for k, name in enumerate(PROF_NAMES)}

    def adjoint_bytes(self) -> int:
        return int(self.lib.fftevp_adjoint_bytes(self.h))

    def adjoint_increment(self, before, after, dL_dSigma, adj, dtheta, opts: Opts | None = None):
        g = (C.c_double * 6)(*[float(x) for x in dL_dSigma])
        th = (C.c_double * 4)(*[float(x) for x in dtheta])
        self._check(self.lib.fftevp_adjoint_increment(
            self.h, C.byref(_opts(opts)), C.c_void_p(before.data_ptr()), C.c_void_p(after.data_ptr()),
            g, C.c_void_p(adj.data_ptr()), th))
        return np.array(th[:])


class PhaseField:
    """Phase-field growth of recrystallised grains (include/fftevp_pf.h) on
    the grid that refines an ``shape`` (n0, n1, n2) mechanical grid 2:1."""

    def __init__(self, shape, K: int = 6, threshold: float = 1e-5, precision: str = "fp64", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("fftevp needs a GPU; no CPU fallback exists")
        self.torch = torch
        self.lib = library()
        self.shape = tuple(int(s) for s in shape)
        self.nvox = int(np.prod(self.shape))
        self.nfine = 8 * self.nvox
        self.K = int(K)
        self.stream = stream or torch.cuda.current_stream()
        prec = {"fp64": FP64, "mixed": MIXED}[precision]
        h = C.c_void_p()
        st = self.lib.fftevp_pf_create(*self.shape, self.K, float(threshold), prec,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != OK:
            raise FftevpError(st, self.lib.fftevp_status_string(st).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.fftevp_pf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != OK:
            raise FftevpError(st, self.lib.fftevp_pf_last_error(self.h).decode())

    def _t(self, a, dtype, n):
        t = self.torch.as_tensor(np.asarray(a) if not self.torch.is_tensor(a) else a, dtype=dtype,
                                 device="cuda").reshape(-1).contiguous()
        if t.numel() != n:
            raise ValueError(f"expected {n} values, got {t.numel()}")
        return t

    def refine(self, grains, estore):
        """Sharp start from a grain map and stored energy on the mechanical grid."""
        g = self._t(grains, self.torch.int32, self.nvox)
        e = self._t(estore, self.torch.float64, self.nvox)
        self._check(self.lib.fftevp_pf_refine(self.h, C.c_void_p(g.data_ptr()), C.c_void_p(e.data_ptr())))

    def load(self, keys, vals, estore):
        """State from slot-major (kin, Vf) keys and values and a fine stored energy."""
        kin = int(np.shape(keys)[0])
        k = self._t(keys, self.torch.int32, kin * self.nfine)
        v = self._t(vals, self.torch.float64, kin * self.nfine)
        e = self._t(estore, self.torch.float64, self.nfine)
        self._check(self.lib.fftevp_pf_import(self.h, C.c_void_p(k.data_ptr()), C.c_void_p(v.data_ptr()),
                                              kin, C.c_void_p(e.data_ptr())))

    def steps(self, n: int):
        self._check(self.lib.fftevp_pf_steps(self.h, int(n)))

    def state(self):
        """(keys int32 (K, Vf), values float64 (K, Vf)) on the device."""
        k = self.torch.empty((self.K, self.nfine), dtype=self.torch.int32, device="cuda")
        v = self.torch.empty((self.K, self.nfine), dtype=self.torch.float64, device="cuda")
        self._check(self.lib.fftevp_pf_export(self.h, C.c_void_p(k.data_ptr()), C.c_void_p(v.data_ptr())))
        return k, v

    def grains(self, before):
        """Grain map on the mechanical grid read from the state."""
        b = self._t(before, self.torch.int32, self.nvox)
        out = self.torch.empty_like(b)
        self._check(self.lib.fftevp_pf_grains(self.h, C.c_void_p(b.data_ptr()), C.c_void_p(out.data_ptr())))
        return out
