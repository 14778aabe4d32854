"""Lattice rotation after each increment (reading of Sec. 2.5, oracle.rotation)
on the GPU against the oracle through the C ABI: orientations and fields over
several increments with both flow laws, mixed precision, snapshots and the
error paths."""
import numpy as np
import pytest

import synth
from oracle import Oracle, Loading
from oracle import ma_roters as OMR

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300))


def qdiff(a, b):
    """Largest difference of quaternion fields (4, V), up to the sign of each."""
    return float(np.minimum(np.abs(a - b).max(axis=0), np.abs(a + b).max(axis=0)).max())


def setup(shape, law, seed, precision="fp64"):
    from paper_1509_04953_amd import Solver, Material, MaRoters, Load
    g = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]
    grains = synth.voronoi_grains(shape, 8, g[0])
    q = synth.random_quaternions(8, g[1])
    quat = np.moveaxis(q[grains], -1, 0).reshape(4, -1).copy()
    rho = synth.lognormal_rho(shape, 2.5e12, 0.3, g[2]).reshape(-1)
    s = Solver(shape, precision)
    s.set_material(Material())
    s.set_microstructure(quat, rho)
    s.set_loading(Load())
    o = Oracle(shape, quat, rho)
    if law == "paper":
        s.set_gnd(grains.reshape(-1))
        o.enable_gnd(grains.reshape(-1), 21.4e-6, 200.0)
        s.set_law(MaRoters())
        o.enable_mr(OMR.MaRoters())
    return s, o, quat


@pytest.mark.parametrize("law,shape,incs", [("power", (16, 16, 16), 3), ("paper", (16, 8, 32), 2)])
def test_rotation_matches_oracle(require_gpu, law, shape, incs):
    from paper_1509_04953_amd import Opts
    s, o, quat0 = setup(shape, law, 81)
    s.set_rotation(True)
    o.enable_rotation()
    for inc in range(incs):
        print(f"case: rotation {law} {shape} increment {inc}", flush=True)
        r = s.step(Opts(tol=1e-11, max_iter=3000))
        ro = o.increment(Loading(), tol=1e-11, max_iter=3000)
        assert r.status == 0 and r.iters == ro["iters"], (r.iters, ro["iters"])
    qg = s.field("quat").cpu().numpy()
    qo = o.field("quat")
    turned = qdiff(qo, quat0)
    print(f"largest orientation change {turned:.2e}, GPU vs oracle {qdiff(qg, qo):.2e}")
    assert turned > 1e-6
    assert qdiff(qg, qo) < 1e-12
    for k in ("sigma", "epsp", "rho"):
        assert rel(s.field(k).cpu().numpy(), o.field(k)) < 1e-10, k


def test_rotation_mixed_and_off(require_gpu):
    from paper_1509_04953_amd import Opts
    s, o, quat0 = setup((16, 16, 16), "power", 82, "mixed")
    s.step(Opts(tol=1e-6))
    assert np.abs(s.field("quat").cpu().numpy() - quat0).max() < 1e-7   # off: unchanged (FP32 copy)
    s.set_rotation(True)
    o.increment(Loading(), tol=1e-6, max_iter=3000)
    o.enable_rotation()
    s.step(Opts(tol=1e-6))
    o.increment(Loading(), tol=1e-6, max_iter=3000)
    assert qdiff(s.field("quat").cpu().numpy(), o.field("quat")) < 1e-5


def test_rotation_snapshots_and_errors(require_gpu):
    import torch
    from paper_1509_04953_amd import Opts, FftevpError, EINVAL
    s, _, _ = setup((16, 16, 16), "power", 83)
    plain = s.save_state()
    s.set_rotation(True)
    with pytest.raises(FftevpError) as e:
        s.load_state(plain)                      # saved without orientations
    assert e.value.status == EINVAL
    s.step(Opts(tol=1e-10))
    snap = s.save_state()
    s.step(Opts(tol=1e-10))
    q2, s2 = s.field("quat").cpu().numpy(), s.field("sigma").cpu().numpy()
    s.load_state(snap)
    s.step(Opts(tol=1e-10))
    assert np.array_equal(q2, s.field("quat").cpu().numpy())
    assert np.array_equal(s2, s.field("sigma").cpu().numpy())
    adj = torch.zeros(s.adjoint_bytes(), dtype=torch.uint8, device="cuda")
    with pytest.raises(FftevpError) as e:
        s.adjoint_increment(snap, s.save_state(), [0, 0, 1, 0, 0, 0], adj, [0, 0, 0, 0])
    assert e.value.status == EINVAL
    assert s.lib.fftevp_set_rotation(s.h, 2) == EINVAL
