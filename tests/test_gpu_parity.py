"""GPU path against the CPU oracle through the C ABI (parity, FP64).

The bar: every field and the mean-stress curve within 1e-10 relative of the
oracle (relative to the field's maximum magnitude), at a tight stop
tolerance; iterates after a fixed number of iterations compare the same way.
"""
import numpy as np
import pytest

import synth
from oracle import Oracle, Loading
from oracle.tensors import voigt_to_mandel

pytestmark = pytest.mark.gpu

TOL_REL = 1e-10


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def gpu_solver(shape, quat, rho, precision="fp64"):
    from paper_1509_04953_amd import Solver, Material, Load
    s = Solver(shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load())
    return s


def micro(shape, n_grains, seed, lognormal=True):
    g_c, g_q, g_r, _ = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]
    grains = synth.voronoi_grains(shape, n_grains, g_c)
    q = synth.random_quaternions(n_grains, g_q)
    quat = np.moveaxis(q[grains], -1, 0).reshape(4, -1).copy()
    rho = (synth.lognormal_rho(shape, 1e12, 0.3, g_r) if lognormal
           else np.full(grains.shape, 1e12)).reshape(-1)
    return quat, rho


def oracle_fields(o):
    return {k: o.field(k) for k in ("sigma", "strain", "epsp", "rho", "gdot")}


def test_first_iterate_matches_local_solve(require_gpu):
    shape = (16, 16, 16)
    quat, rho = micro(shape, 8, 11)
    from paper_1509_04953_amd import Opts
    s = gpu_solver(shape, quat, rho)
    print("case: first iterate 16^3", flush=True)
    rep = s.step(Opts(tol=1e-14, max_iter=1))
    assert rep.status == 1 and rep.iters == 1
    o = Oracle(shape, quat, rho)
    orep = o.increment(Loading(), tol=1e-14, max_iter=1)
    sg = s.field("sigma_iter").cpu().numpy()
    assert rel(sg, o.field("sigma")) < TOL_REL
    np.testing.assert_allclose(rep.Sigma, orep["Sigma"], rtol=1e-11, atol=1e-9)


# every line length the transforms support along each axis (radix plans
# 8, 16, 8x4, 8x8, 16x8, 16x16, 8x8x8; 512 voxels per x-line takes the
# local kernel's two-voxels-per-thread path)
@pytest.mark.parametrize("shape,k", [((16, 16, 16), 3), ((32, 8, 16), 4), ((8, 32, 16), 2),
                                     ((8, 8, 8), 3), ((64, 16, 128), 2),
                                     ((256, 8, 8), 3), ((8, 256, 8), 3), ((8, 8, 256), 3),
                                     ((512, 8, 8), 3), ((8, 512, 8), 3), ((8, 8, 512), 3)])
def test_iterates_match(require_gpu, shape, k):
    quat, rho = micro(shape, 6, 12)
    from paper_1509_04953_amd import Opts
    s = gpu_solver(shape, quat, rho)
    print(f"case: iterates {shape} k={k}", flush=True)
    rep = s.step(Opts(tol=1e-14, max_iter=k))
    assert rep.iters == k
    o = Oracle(shape, quat, rho)
    orep = o.increment(Loading(), tol=1e-14, max_iter=k)
    assert rel(s.field("sigma_iter").cpu().numpy(), o.field("sigma")) < TOL_REL
    assert rel(s.field("strain_iter").cpu().numpy(), o.field("strain")) < TOL_REL
    assert abs(rep.err_c - orep["err_c"]) <= 1e-8 * orep["err_c"]
    np.testing.assert_allclose(rep.E, orep["E"], rtol=1e-10, atol=1e-16)


# FP32 fields on lines of 256 points: the z and inverse y passes take tiles
# of four x-frequencies there and move pairs of lines per 16-byte access. The
# FP32 Newton solve stops at a 1e-5 relative step, so unconverged iterates
# carry errors of that order (observed 7e-6 stress, 1.8e-5 strain); a wrong
# tile or pair mapping gives O(1).
@pytest.mark.parametrize("shape", [(16, 256, 8), (16, 8, 256), (256, 8, 8)])
def test_iterates_match_mixed(require_gpu, shape):
    quat, rho = micro(shape, 6, 13)
    from paper_1509_04953_amd import Opts
    s = gpu_solver(shape, quat, rho, "mixed")
    print(f"case: mixed iterates {shape}", flush=True)
    rep = s.step(Opts(tol=1e-14, max_iter=3))
    assert rep.iters == 3
    o = Oracle(shape, quat, rho)
    o.increment(Loading(), tol=1e-14, max_iter=3)
    for k, v in (("sigma_iter", o.field("sigma")), ("strain_iter", o.field("strain"))):
        err = rel(s.field(k).cpu().numpy(), v)
        print(k, err, flush=True)
        assert err < 5e-5, (k, err)


def test_increments_tight(require_gpu):
    w = synth.workload("cu16")
    quat, rho, _ = synth.make_microstructure(w)
    quat = quat.reshape(4, -1)
    from paper_1509_04953_amd import Opts
    s = gpu_solver(w.shape, quat, rho.reshape(-1))
    o = Oracle(w.shape, quat, rho)
    for inc in range(3):
        print(f"case: cu16 increment {inc}", flush=True)
        rep = s.step(Opts(tol=1e-12, max_iter=2000))
        orep = o.increment(Loading(), tol=1e-12, max_iter=2000)
        assert rep.status == 0, rep
        assert abs(rep.iters - orep["iters"]) <= 1
        assert rel(rep.Sigma[2], orep["Sigma"][2]) < TOL_REL
        for k, v in oracle_fields(o).items():
            g = s.field(k).cpu().numpy()
            assert rel(g, v) < TOL_REL, (inc, k, rel(g, v))
