"""fftevp_step_noalloc (the increment with its scratch in the library's
static device array) against fftevp_step, through the C ABI: two calls in a
row, the second on a smaller grid, each bit-identical to the allocating
entry point on a twin context; and the size limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def twin(shape, precision, seed):
    from paper_1509_04953_amd import Solver, Material, Load
    g = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]
    grains = synth.voronoi_grains(shape, 6, g[0])
    q = synth.random_quaternions(6, g[1])
    quat = np.moveaxis(q[grains], -1, 0).reshape(4, -1).copy()
    rho = synth.lognormal_rho(shape, 1e12, 0.3, g[2]).reshape(-1)
    out = []
    for _ in range(2):
        s = Solver(shape, precision)
        s.set_material(Material())
        s.set_microstructure(quat, rho)
        s.set_loading(Load())
        out.append(s)
    return out


def fields(s):
    return {k: s.field(k).cpu().numpy() for k in ("sigma", "strain", "epsp", "rho")}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_noalloc_matches_step(require_gpu, precision):
    from paper_1509_04953_amd import Opts
    opts = Opts(tol=1e-8 if precision == "fp64" else 1e-6, max_iter=3000)
    for shape, seed in (((32, 32, 16), 5), ((16, 8, 8), 6)):     # second call: smaller grid
        print(f"case: step_noalloc {precision} {shape}", flush=True)
        ref, na = twin(shape, precision, seed)
        for inc in range(2):
            r1 = ref.step(opts)
            r2 = na.step_noalloc(opts)
            assert r1.status == r2.status == 0
            assert r1.iters == r2.iters and r1.newton_failed == r2.newton_failed
            assert np.array_equal(r1.Sigma, r2.Sigma) and np.array_equal(r1.E, r2.E)
            assert r1.rho_mean == r2.rho_mean and r1.err_c == r2.err_c
        f1, f2 = fields(ref), fields(na)
        for k in f1:
            assert np.array_equal(f1[k], f2[k]), k
        ref.close()
        na.close()


def test_step_noalloc_size_limit(require_gpu):
    from paper_1509_04953_amd import Solver, Material, Load, FftevpError, EINVAL
    print("case: step_noalloc size limit 256x256x512 mixed", flush=True)
    s = Solver((256, 256, 512), "mixed")
    with pytest.raises(FftevpError) as e:
        s.step_noalloc()
    assert e.value.status == EINVAL
    s.close()
