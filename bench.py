"""Benchmark: FFT-EVP voxel-iterations/s on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cu128]

A step is one strain increment of the synthetic 128^3 copper polycrystal
(500 periodic Voronoi grains, uniformly random orientations, log-normal
dislocation density, uniaxial compression at 1e-3/s in increments of 2e-3,
stop tolerance 1e-6): the whole fixed-point solve (local Newton + x-FFTs,
reduction and stop test, y/z FFTs with the Green operator) and the
end-of-increment state update. W untimed increments come first, then K timed
ones. The FP64 path gives ``value``; the mixed-precision path (FP32 fields,
transforms and Newton; FP64 reductions and macroscopic update) is timed the
same way and reported under ``mixed``. ``adjoint`` reports the wall time of
the curve-loss gradient (backward, with segment recomputation from the
checkpoints of the memory-aware schedule: every increment's state when all
fit in half of the free device memory) over that of the forward pass, on the
128^3 / 300-grain / 40-increment workload.

voxel-iterations/s = sum over timed increments of (fixed-point iterations x
voxels) / wall time, with inputs resident in HBM. Per-kernel durations come
from HIP events the library records around each launch on its stream.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_bytes(shape, word):
    """Algorithmic HBM bytes per launch of each solver kernel."""
    n0, n1, n2 = shape
    V = n0 * n1 * n2
    planes = n1 * n2
    return {
        # e spectra 6, lam 6, epsp 6, rho 1, quat 4 in; sigma 6, tau spectra 6 out
        "local": (35 * V + 12 * planes) * word,
        "yfwd": 12 * V * word,
        "zgamma": 12 * V * word,
        "yinv": 12 * V * word,
    }


def run_gpu(w, quat, rho, precision, steps, warmup):
    """Timed increments; HIP events bracket only the local kernel during the
    timed region (events cost ~4 us per launch), then two more increments
    are run with every kernel class timed for the per-kernel table."""
    import torch
    from paper_1509_04953_amd import Solver, Material, Load, Opts
    s = Solver(w.shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load(dt=w.dt))
    opts = Opts(tol=w.tol, max_iter=2000)
    for k in range(warmup):
        r = s.step(opts)
        print(f"# {precision} warmup {k}: iters {r.iters} s33 {r.Sigma[2]:.4f}", file=sys.stderr, flush=True)
    s.set_profiling(True, classes=("local",))
    s.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    s33 = []
    newton = []
    for k in range(steps):
        r = s.step(opts)
        iters.append(r.iters)
        s33.append(r.Sigma[2])
        newton.append(r.newton_mean)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = s.profile(reset=True)
    s.set_profiling(True)
    for k in range(2):
        s.step(opts)
    torch.cuda.synchronize()
    prof_all = s.profile(reset=True)
    s.close()
    print(f"# {precision}: {steps} increments, {sum(iters)} iterations, {dt:.3f} s", file=sys.stderr, flush=True)
    return dict(time=dt, iters=iters, s33=s33, prof=prof, prof_all=prof_all, newton_mean=float(np.mean(newton)),
                rate=sum(iters) * w.voxels / dt, ms_per_step=1e3 * dt / steps)


def run_adjoint(w, quat, rho, precision, increments=None):
    """Forward and backward wall time of the curve-loss gradient."""
    import torch
    from paper_1509_04953_amd import Solver, Material, Load, Opts
    from paper_1509_04953_amd.adjoint import CurveProblem, StressStrainCurve, curve_loss
    T = increments or w.increments
    s = Solver(w.shape, precision)
    opts = Opts(tol=w.tol, max_iter=2000)
    p = CurveProblem(s, Material(), quat, rho, Load(dt=w.dt), T, opts, opts)
    torch.cuda.reset_peak_memory_stats()
    th = torch.tensor(Material().theta(), dtype=torch.float64, requires_grad=True)
    tgt = torch.zeros(T, dtype=torch.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c = StressStrainCurve.apply(th, p)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # target: the curve of parameters theta0 * (1.05, 0.95, 1.05, 0.95) would need a
    # second forward; the timing does not depend on the target values
    L = curve_loss(c, tgt + c.detach() * 1.01)
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.close()
    print(f"# adjoint {precision}: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s", file=sys.stderr,
          flush=True)
    its = int(sum(p.iterations))
    return {"workload": f"{w.shape[0]}^3, {w.n_grains} grains, {T} increments",
            "precision": precision, "forward_s": t1 - t0, "backward_s": t2 - t1,
            "adjoint_over_forward": (t2 - t1) / (t1 - t0),
            "checkpoint_every": int(p.schedule),
            "forward_iterations": its,
            "forward_voxel_iterations_per_s": its * w.voxels / (t1 - t0),
            "final_strain": -w.d_eps * T, "s33_final": float(c.detach()[-1]),
            "peak_mem_GB": torch.cuda.max_memory_allocated() / 1e9,
            "grad": th.grad.numpy().tolist()}


def run_gnd(w, quat, rho, grains, precision, increments=4):
    """GND update (grain-aware slip-rate gradients, Sec. 2.2 Eq. 7-8) on the
    same workload: HIP-event time of the GND kernel per increment and its HBM
    roofline."""
    from paper_1509_04953_amd import Solver, Material, Load, Opts
    s = Solver(w.shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load(dt=w.dt))
    s.set_gnd(grains.reshape(-1))
    opts = Opts(tol=w.tol, max_iter=2000)
    s.step(opts)
    s.set_profiling(True, classes=("gnd",))
    s.profile(reset=True)
    for _ in range(increments):
        r = s.step(opts)
    ms, n = s.profile(reset=True)["gnd"]
    s.close()
    word = 8 if precision == "fp64" else 4
    V = w.voxels
    # the GND kernel: slip rates 12, orientation 4, densities 24 in (+ int32
    # grain id), densities 24 out (the state update writes the 12 rates)
    nbytes = 64 * V * word + 4 * V
    avg = ms / max(n, 1)
    gbs = nbytes / (avg * 1e-3) / 1e9
    return {"precision": precision, "ms_per_increment": avg, "increments": n,
            "bytes_per_increment": nbytes, "GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
            "l_eff_m": r.l_eff}


def run_rotation(w, quat, rho, precision, increments=4):
    """Lattice rotation after each increment (k_rotate): HIP-event time per
    increment and the rate of its algorithmic bytes (slip rates 12 words and
    orientation 4 words read, orientation 4 words written per voxel)."""
    from paper_1509_04953_amd import Solver, Material, Load, Opts
    s = Solver(w.shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load(dt=w.dt))
    s.set_rotation(True)
    s.set_profiling(True, classes=("rotate",))
    s.profile(reset=True)
    for _ in range(increments):
        s.step(Opts(tol=w.tol, max_iter=2000))
    ms, n = s.profile(reset=True)["rotate"]
    s.close()
    word = 8 if precision == "fp64" else 4
    nbytes = 20 * w.voxels * word
    avg = ms / max(n, 1)
    return {"precision": precision, "ms_per_increment": avg, "increments": n,
            "GBps": nbytes / (avg * 1e-3) / 1e9, "frac_hbm": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS}


def run_mr(w, quat, rho, precision, steps=3, warmup=1):
    """The paper's own flow rule and SSD evolution (Sec. 2.2, Eq. 3-6) on the
    same workload (initial SSD density 2.5e12 m^-2 per voxel scaled by the
    workload's log-normal field): voxel-iterations/s, iterations per
    increment and the local kernel's HBM rate. Its algorithmic bytes per
    voxel: the power-law kernel's 35 words minus the density plus 36 words of
    per-system parameters (tau_pass, 1/tau_cut, prefactor)."""
    import torch
    from paper_1509_04953_amd import Solver, Material, MaRoters, Load, Opts
    s = Solver(w.shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho * 2.5)
    s.set_loading(Load(dt=w.dt))
    s.set_law(MaRoters())
    opts = Opts(tol=w.tol, max_iter=3000)
    for _ in range(warmup):
        s.step(opts)
    s.set_profiling(True, classes=("local",))
    s.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(steps):
        r = s.step(opts)
        iters.append(r.iters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = s.profile(reset=True)["local"]
    s.close()
    word = 8 if precision == "fp64" else 4
    nbytes = (35 - 1 + 36) * w.voxels * word + 12 * w.shape[1] * w.shape[2] * word
    avg = ms / max(n, 1)
    return {"precision": precision, "value": sum(iters) * w.voxels / dt, "unit": "voxel-iterations/s",
            "iters_per_increment": float(np.mean(iters)), "s33_last": float(r.Sigma[2]),
            "local_avg_ms": avg, "local_GBps": nbytes / (avg * 1e-3) / 1e9,
            "local_frac_hbm": nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS}


def run_drx(w, quat, rho, grains, precision, tests=4):
    """DRX nucleation test (Sec. 2.3, 2.5) on the same workload after one
    increment with GND tracking: wall time per test with the uniforms
    already on the device (validation pass + nucleation kernel + count)."""
    import torch
    from paper_1509_04953_amd import Solver, Material, Load, Opts
    s = Solver(w.shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load(dt=w.dt))
    s.set_gnd(grains.reshape(-1))
    gen = torch.Generator(device="cuda").manual_seed(0)
    u = torch.rand(w.voxels, dtype=torch.float64, device="cuda", generator=gen)
    s.set_drx(u, kc=2.0e12)
    s.step(Opts(tol=w.tol, max_iter=2000))
    us = [torch.rand(w.voxels, dtype=torch.float64, device="cuda", generator=gen) for _ in range(tests)]
    torch.cuda.synchronize()
    n = []
    t0 = time.perf_counter()
    for u in us:
        n.append(s.drx_nucleate(u))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / tests
    s.close()
    return {"precision": precision, "ms_per_test": dt * 1e3, "nuclei": n}


def run_coupled(w, quat, rho, grains, precision, cycles=3, pf_steps=20):
    """The coupled loop (Sec. 2.5) on the workload: per increment the
    mechanical solve with GND tracking, the nucleation test, pf_steps
    phase-field steps on the 2:1 grid with the grain map written back, and
    the stress redistribution (the increment's solve repeated with the
    updated microstructure). Host
    wall time per phase (each phase ends with a synchronisation), stored
    energy at a PF spacing of 1 mm so that nuclei grow."""
    import torch
    from paper_1509_04953_amd import Solver, PhaseField, Material, Load, Opts
    s = Solver(w.shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load(dt=w.dt))
    s.set_gnd(grains.reshape(-1))
    gen = torch.Generator(device="cuda").manual_seed(1)
    s.set_drx(torch.rand(w.voxels, dtype=torch.float64, device="cuda", generator=gen), kc=4.0e12)
    pf = PhaseField(w.shape, K=6, threshold=1e-5, precision=precision)
    opts = Opts(tol=w.tol, max_iter=2000)
    t = {"solve": 0.0, "nucleate": 0.0, "grow": 0.0, "redistribute": 0.0}
    log = []
    for _ in range(cycles):
        u = torch.rand(w.voxels, dtype=torch.float64, device="cuda", generator=gen)
        before = s.save_state()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.step(opts)
        t1 = time.perf_counter()
        n = s.drx_nucleate(u)
        t2 = time.perf_counter()
        ch, rex = s.drx_grow(pf, pf_steps, dx=1.0e-3)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rr = s.redistribute(before, opts)
        t4 = time.perf_counter()
        t["solve"] += t1 - t0
        t["nucleate"] += t2 - t1
        t["grow"] += t3 - t2
        t["redistribute"] += t4 - t3
        log.append({"iters": r.iters, "nuclei": n, "changed": ch, "recrystallised": rex,
                    "redistribution_iters": rr.iters, "s33": r.Sigma[2], "s33_redistributed": rr.Sigma[2]})
    pf.close()
    s.close()
    return {"precision": precision, "cycles": cycles, "pf_steps": pf_steps,
            "ms_per_cycle": {k: v / cycles * 1e3 for k, v in t.items()}, "log": log}


def run_pf(w, grains, precision, steps=200, warmup=100, K=6):
    """Phase-field grain growth (Sec. 2.4) on the 2:1 grid of the workload
    (one PF point per eighth of a voxel): grain map with one-voxel nuclei on
    5% of the boundary voxels, stored energy log-normal with median 0.7 in
    PF units (rho_tot ~ 1e14 m^-2 at the paper's voxel size). ``warmup``
    steps let the sharp boundaries relax first; then ``steps`` steps are
    timed with HIP events on the stream the kernels run on. Algorithmic
    bytes per step: per point, the count byte and the used (key, value)
    slots read and written once, plus the stored energy where both kinds of
    order parameter meet (the only points that read it)."""
    import torch
    import synth
    from paper_1509_04953_amd import PhaseField
    rng = np.random.default_rng(w.seed + 1000)
    g = synth.single_voxel_nuclei(grains, 0.05, rng).reshape(-1)
    E = synth.lognormal_rho(w.shape, 0.7, 0.3, rng).reshape(-1)
    pf = PhaseField(w.shape, K=K, threshold=1e-5, precision=precision)
    pf.refine(g, E)
    pf.steps(warmup)
    k, v = pf.state()
    used = v > 0
    c = used.sum(0).double()
    rex = (used & ((k & 1) == 1)).any(0)
    dfm = (used & ((k & 1) == 0)).any(0)
    word = 8 if precision == "fp64" else 4
    nbytes = float(2 * (1 + c * (4 + word)).sum() + word * (rex & dfm).sum())
    mean_slots = float(c.mean())
    del k, v, used, c, rex, dfm
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    pf.steps(steps)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gbs = nbytes / (ms * 1e-3) / 1e9
    pf.close()
    summary = "phasefield_256cube_k_pf_step.md"
    full = w.shape == (128, 128, 128) and K == 6
    prec = "fp64" if precision == "fp64" else "mixed"
    issue = stored_valu_issue_us("k_pf_step", prec, summary, PF_SOURCES) if full else None
    return {"precision": precision, "pf_points": 8 * w.voxels, "K": K, "steps": steps,
            "warmup_steps": warmup, "ms_per_step": ms,
            "point_steps_per_s": 8 * w.voxels / (ms * 1e-3), "mean_slots_per_point": mean_slots,
            "roofline": {"kernel": "k_pf_step", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "bytes_per_step": nbytes,
                         "traffic": stored_traffic("k_pf_step", prec, summary, PF_SOURCES) if full else None,
                         # limited by vector-ALU issue (candidate matching), not by HBM
                         "valu_issue_frac": (issue * 1e-3 / ms) if issue else None}}


FFTEVP_SOURCES = ("kernels.hip", "device_math.h", "fft_lds.h")
PF_SOURCES = ("phasefield.hip",)


def source_hash(files=FFTEVP_SOURCES):
    """Prefix of the sha256 of device sources (matches the profiles)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1509_04953_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, precision, summary="fftevp_128cube_hbm_traffic.md", files=FFTEVP_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    src = source_hash(files)
    for ln in lines:
        f = ln.split()
        if len(f) >= 3 and f[0] == "traffic" and f[1] == kernel and f[2] == precision:
            kv = dict(x.split("=", 1) for x in f[3:])
            if kv.get("sources") != src:
                return None
            return (float(kv["fetch_kib"]) * float(kv["fetch_factor"])
                    + float(kv["write_kib"]) * float(kv["write_factor"])) * 1024.0
    return None


def stored_valu_issue_us(kernel, precision, summary="fftevp_128cube_sq_counters.md", files=FFTEVP_SOURCES):
    """VALU issue time per launch (us) from the committed shader-counter
    summary: SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x 2.4 GHz); None when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    src = source_hash(files)
    for ln in lines:
        f = ln.split()
        if len(f) >= 3 and f[0] == "valu" and f[1] == kernel and f[2] == precision:
            kv = dict(x.split("=", 1) for x in f[3:])
            return float(kv["issue_us"]) if kv.get("sources") == src else None
    return None


def roofline(w, res, word):
    """Roofline of the local kernel (the dominant one) from the timed region;
    per-kernel averages from the fully timed follow-up increments."""
    by = kernel_bytes(w.shape, word)
    ms, n = res["prof"]["local"]
    avg = ms / max(n, 1)
    achieved = by["local"] / (avg * 1e-3) / 1e9
    pa = res["prof_all"]
    per_kernel = {k: {"avg_ms": pa[k][0] / max(pa[k][1], 1), "launches": pa[k][1],
                      "GBps": by[k] / (pa[k][0] / max(pa[k][1], 1) * 1e-3) / 1e9}
                  for k in by}
    share = {k: pa[k][0] for k in by}
    dom = max(share, key=share.get)
    prec = "fp64" if word == 8 else "mixed"
    issue = stored_valu_issue_us("k_local", prec) if w.shape == (128, 128, 128) else None
    return {"kernel": "local", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": stored_traffic("k_local", prec) if w.shape == (128, 128, 128) else None,
            "bytes_per_launch": by["local"], "avg_ms": avg, "launches": n,
            "largest_share": dom,
            # the local kernel is limited by its vector-ALU issue rate: the
            # profiled VALU issue time over this run's average launch time
            "valu_issue_frac": (issue * 1e-3 / avg) if issue else None}, per_kernel


def _cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, quat, rho, n=24):
    """The oracle as written, timed on the host on a bounded sample of the
    same workload: the whole first increment (every fixed-point iteration,
    to the workload's tolerance) on an n^3 window cut from its
    microstructure (same grains, orientations and density field; one
    full-grid iteration of the 128^3 oracle alone takes minutes), with the
    oracle's own increment code, excluding the one-off Green-operator set-up.
    Timed twice: with numpy's default thread pools (every host core
    available) and limited to one thread."""
    from threadpoolctl import threadpool_limits
    from oracle import Oracle, Loading
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    q = np.ascontiguousarray(quat.reshape(4, w.shape[2], w.shape[1], w.shape[0])[:, :n, :n, :n]).reshape(4, -1)
    r = np.ascontiguousarray(rho.reshape(w.shape[2], w.shape[1], w.shape[0])[:n, :n, :n]).reshape(-1)
    runs = {}
    for label, limit in (("all_cores", None), ("one_core", 1)):
        o = Oracle((n, n, n), q, r)
        o.spectral_update(np.zeros((o.nvox, 6)), np.zeros(6))   # Green operator set-up, untimed
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            rep = o.increment(Loading(dt=w.dt), tol=w.tol, max_iter=2000)
            dt = time.perf_counter() - t0
        runs[label] = {"seconds": dt, "iterations": rep["iters"],
                       "voxel_iterations_per_s": rep["iters"] * o.nvox / dt,
                       "threads": nproc if limit is None else 1}
        print(f"# cpu baseline {label}: {rep['iters']} iterations, {dt:.1f} s", file=sys.stderr, flush=True)
    best = max(runs.values(), key=lambda x: x["voxel_iterations_per_s"])
    return {"value": best["voxel_iterations_per_s"], "unit": "voxel-iterations/s",
            "cores": best["threads"], "kind": "oracle",
            "sample": f"the whole first increment (tol {w.tol}) on a {n}^3 window of the {w.shape[0]}^3 "
                      f"workload's microstructure, the oracle's increment code (numpy FP64), "
                      f"Green-operator set-up excluded",
            "nproc": nproc, "cpu_model": _cpu_model(), "runs": runs}


def run_cu256(precision="mixed", increments=200):
    """The largest workload (256^3, 2000 grains, log-normal density with 5 %
    low-density grain-boundary nuclei): the stress-strain curve over the
    whole path (200 increments to 40 % compression) with its adjoint
    gradient from ceil(sqrt(200)) = 15-increment checkpoints. Forward rate,
    adjoint/forward wall time, peak device memory."""
    import synth
    w = synth.workload("cu256")
    t0 = time.perf_counter()
    quat, rho, _ = synth.make_microstructure(w)
    print(f"# cu256 microstructure {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return run_adjoint(w, quat.reshape(4, -1), rho.reshape(-1), precision, increments)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cu128")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-gnd", action="store_true")
    ap.add_argument("--no-mr", action="store_true")
    ap.add_argument("--no-pf", action="store_true")
    ap.add_argument("--no-cu256", action="store_true",
                    help="skip the 256^3 whole-path mixed-precision curve and adjoint")
    ap.add_argument("--cu256-increments", type=int, default=200)
    ap.add_argument("--adjoint-workload", default="cu128adj")
    ap.add_argument("--adjoint-increments", type=int, default=0,
                    help="increments of the adjoint run (default: the workload's)")
    ap.add_argument("--adjoint-precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solve is built and measured for a single MI355X; "
              "multi-GPU sharding is a design note only.", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": a.numel() * 8, "copies": 3}))
        return
    w = synth.workload(args.workload)
    quat, rho, grains = synth.make_microstructure(w)
    quat = quat.reshape(4, -1)
    rho = rho.reshape(-1)
    out = {}
    precs = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    for p in precs:
        out[p] = run_gpu(w, quat, rho, p, args.steps, args.warmup)
    main_p = precs[0]
    r = out[main_p]
    word = 8 if main_p == "fp64" else 4
    roof, per_kernel = roofline(w, r, word)
    line = {
        "metric": "FFT-EVP voxel-iterations/s at 128\u00b3 (FP64 vs mixed), adjoint/forward time",
        "grid": list(w.shape),
        "value": r["rate"],
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{w.shape[0]}x{w.shape[1]}x{w.shape[2]} Cu polycrystal, "
                               f"{w.n_grains} Voronoi grains, log-normal rho, uniaxial compression, "
                               f"d_eps {w.d_eps}, tol {w.tol}",
                   "precision": main_p, "iterations": sum(r["iters"]),
                   "mean_iters_per_increment": float(np.mean(r["iters"])),
                   "newton_per_voxel": r["newton_mean"]},
        "roofline": roof,
        "kernels": per_kernel,
    }
    if "mixed" in out and main_p != "mixed":
        m = out["mixed"]
        mroof, mk = roofline(w, m, 4)
        line["mixed"] = {"value": m["rate"], "ms_per_step": m["ms_per_step"],
                         "iterations": sum(m["iters"]), "roofline": mroof, "kernels": mk,
                         "s33_rel_diff_vs_fp64": float(np.max(np.abs(np.array(m["s33"]) - np.array(r["s33"])))
                                                       / np.max(np.abs(r["s33"])))}
    if not args.no_gnd:
        line["gnd"] = run_gnd(w, quat, rho, grains, precs[0])
    if not args.no_gnd:
        line["drx"] = run_drx(w, quat, rho, grains, precs[0])
        line["rotation"] = run_rotation(w, quat, rho, precs[0])
    if not args.no_mr:
        line["paper_law"] = {p: run_mr(w, quat, rho, p) for p in precs}
    if not args.no_pf:
        line["phase_field"] = {p: run_pf(w, grains, p) for p in precs}
    if not args.no_pf and not args.no_gnd:
        line["coupled"] = run_coupled(w, quat, rho, grains, precs[0])
    if not args.no_adjoint:
        wa = synth.workload(args.adjoint_workload)
        if wa.name == w.name:
            qa, ra = quat, rho
        else:
            qa, ra, _ = synth.make_microstructure(wa)
            qa, ra = qa.reshape(4, -1), ra.reshape(-1)
        line["adjoint"] = run_adjoint(wa, qa, ra, args.adjoint_precision, args.adjoint_increments or None)
    if not args.no_cu256:
        line["cu256"] = run_cu256("mixed", args.cu256_increments)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w, quat, rho)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
