"""The paper's own constitutive law (Sec. 2.2, Eq. 3-6) on the GPU against
the oracle, through the C ABI: fields and per-system SSD densities after
whole increments, with and without GND densities in the projections, the
mixed path, snapshots and error paths."""
import numpy as np
import pytest

import synth
from oracle import Oracle, Loading
from oracle import ma_roters as OMR

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def setup(shape, n_grains, seed, precision="fp64", gnd=False):
    from paper_1509_04953_amd import Solver, Material, MaRoters, Load
    g = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]
    grains = synth.voronoi_grains(shape, n_grains, g[0])
    q = synth.random_quaternions(n_grains, g[1])
    quat = np.moveaxis(q[grains], -1, 0).reshape(4, -1).copy()
    rho = synth.lognormal_rho(shape, 2.5e12, 0.3, g[2]).reshape(-1)
    s = Solver(shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load())
    o = Oracle(shape, quat, rho)
    if gnd:
        s.set_gnd(grains.reshape(-1))
        o.enable_gnd(grains.reshape(-1), 21.4e-6, 200.0)
    s.set_law(MaRoters())
    o.enable_mr(OMR.MaRoters())
    return s, o


@pytest.mark.parametrize("shape,gnd", [((16, 16, 16), False), ((16, 8, 32), True)])
def test_paper_law_matches_oracle(require_gpu, shape, gnd):
    from paper_1509_04953_amd import Opts
    s, o = setup(shape, 8, 41, gnd=gnd)
    for inc in range(2):
        print(f"case: paper's law {shape} gnd={gnd} increment {inc}", flush=True)
        r = s.step(Opts(tol=1e-11, max_iter=3000))
        ro = o.increment(Loading(), tol=1e-11, max_iter=3000)
        assert r.status == 0, r
        assert r.iters == ro["iters"], (r.iters, ro["iters"])
        assert abs(r.Sigma[2] - ro["Sigma"][2]) < 1e-10 * abs(ro["Sigma"][2])
        assert abs(r.rho_mean - ro["rho_mean"]) < 1e-10 * ro["rho_mean"]
    names = ["sigma", "strain", "epsp", "rho", "rho_ssd", "gdot"] + (["rho_gnds", "rho_gndet"] if gnd else [])
    for k in names:
        g = s.field(k).cpu().numpy()
        v = o.field(k)
        assert rel(g, v) < 1e-10, (k, rel(g, v))


# Lines of 256 and 512 points run the local kernel in 256-thread blocks,
# which stage two of the three per-system parameter rows in LDS (all three
# in 128-thread blocks, the cases above), and at 512 two voxels per thread.
# Whole increments take the oracle minutes there, so the k-th iterates are
# compared instead.
@pytest.mark.parametrize("shape,precision", [((256, 8, 8), "fp64"), ((512, 8, 8), "fp64"), ((256, 8, 8), "mixed")])
def test_paper_law_iterates_long_lines(require_gpu, shape, precision):
    from paper_1509_04953_amd import Opts
    s, o = setup(shape, 8, 44, precision=precision)
    k = 8
    print(f"case: paper's law iterates {shape} {precision} k={k}", flush=True)
    r = s.step(Opts(tol=1e-14, max_iter=k))
    assert r.iters == k
    ro = o.increment(Loading(), tol=1e-14, max_iter=k)
    bound = 1e-10 if precision == "fp64" else 1e-4
    for name, v in (("sigma_iter", o.field("sigma")), ("strain_iter", o.field("strain"))):
        err = rel(s.field(name).cpu().numpy(), v)
        print(name, err, flush=True)
        assert err < bound, (name, err)
    if precision == "fp64":
        assert abs(r.err_c - ro["err_c"]) <= 1e-8 * ro["err_c"]


def test_paper_law_mixed_precision(require_gpu):
    from paper_1509_04953_amd import Opts
    s, o = setup((16, 16, 16), 8, 42, precision="mixed")
    for inc in range(2):
        print(f"case: paper's law mixed increment {inc}", flush=True)
        s.step(Opts(tol=1e-6))
        o.increment(Loading(), tol=1e-6, max_iter=3000)
    for k in ("sigma", "strain", "epsp", "rho_ssd"):
        g = s.field(k).cpu().numpy()
        v = o.field(k)
        err = np.linalg.norm(g - v) / np.linalg.norm(v)
        print(k, "mixed relative L2 error", err, flush=True)
        assert err < 1e-4, (k, err)


def test_paper_law_snapshots_and_errors(require_gpu):
    from paper_1509_04953_amd import Solver, Material, MaRoters, Opts, FftevpError, EINVAL, ESTATE
    print("case: paper's law snapshots", flush=True)
    s, _ = setup((16, 16, 16), 8, 43)
    o = Opts(tol=1e-8)
    s.step(o)
    snap = s.save_state()
    s.step(o)
    a = [s.field(k).cpu().numpy() for k in ("sigma", "rho_ssd")]
    s.load_state(snap)
    s.step(o)
    b = [s.field(k).cpu().numpy() for k in ("sigma", "rho_ssd")]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # the power-law context refuses the snapshot; adjoint is power-law only
    t = Solver((16, 16, 16))
    with pytest.raises(FftevpError) as e:
        t.load_state(snap)
    assert e.value.status == EINVAL
    with pytest.raises(FftevpError) as e:
        t.set_law(MaRoters())
    assert e.value.status == ESTATE
    t.set_material(Material())
    with pytest.raises(FftevpError) as e:
        t.field("rho_ssd")
    assert e.value.status == ESTATE
    adj = s.torch.zeros(s.adjoint_bytes() // 8 + 1, dtype=s.torch.float64, device="cuda")
    with pytest.raises(FftevpError) as e:
        s.adjoint_increment(snap, snap, np.zeros(6), adj, np.zeros(4))
    assert e.value.status == EINVAL
