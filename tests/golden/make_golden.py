"""Write the stored expected values of the GPU tests. Calls only the oracle.

    python tests/golden/make_golden.py

* adjoint_8cube.json: an 8^3 four-grain polycrystal; the mean-stress curve
  over 3 compression increments at the reference parameters, the target
  curve at perturbed parameters theta* = theta0 * (1.05, 0.95, 1.05, 0.95),
  and the central finite-difference gradient of the curve loss
  L = mean_t (<s33>_t - target_t)^2 with respect to (tau0, k1, k2, n).
* curve_16cube.json: the mean-stress curve of the 16^3 eight-grain
  polycrystal (uniform density) over 5 increments.
Both solve each increment to a stop tolerance of 1e-13.
* curve_64cube.json: the 64^3, 100-grain, log-normal-density polycrystal
  over its first 3 increments at the workload's stop tolerance 1e-6, with
  the iteration counts and sampled fields (slow: about 10 minutes).
* curve_128cube.json: the 128^3, 500-grain, log-normal-density benchmark
  polycrystal over its first increment at the workload's stop tolerance
  1e-6: iteration count, mean stress and strain, and the stress, strain,
  plastic strain and density at 256 sampled voxels (slow: 87 oracle
  iterations of about 3 minutes each, 4.5 hours on one core, and 10 GB of
  memory).
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import Flow, Loading, stress_curve, fd_gradient, curve_loss  # noqa: E402


def adjoint_case():
    w = synth.Workload("adj8", (8, 8, 8), 4, "lognormal", 3, 1e-13, seed=41)
    q, rho, _ = synth.make_microstructure(w)
    f0 = Flow()
    th0 = f0.theta()
    ths = th0 * np.array([1.05, 0.95, 1.05, 0.95])
    load = Loading()
    c0, r0 = stress_curve(w.shape, q, rho, f0, load, w.increments, tol=1e-13)
    cs, _ = stress_curve(w.shape, q, rho, f0.with_theta(ths), load, w.increments, tol=1e-13)
    g = fd_gradient(w.shape, q, rho, f0, load, w.increments, cs, rel_step=1e-5, tol=1e-13)
    return {"workload": {"shape": w.shape, "grains": w.n_grains, "rho": w.rho, "seed": w.seed},
            "theta0": th0.tolist(), "theta_star": ths.tolist(), "increments": w.increments,
            "curve_theta0": c0.tolist(), "target": cs.tolist(), "loss": curve_loss(c0, cs),
            "fd_gradient": g.tolist(), "fd_rel_step": 1e-5, "tol": 1e-13,
            "iters": [r["iters"] for r in r0]}


def curve16():
    w = synth.workload("cu16")
    q, rho, _ = synth.make_microstructure(w)
    c, reps = stress_curve(w.shape, q, rho, Flow(), Loading(), w.increments, tol=1e-13)
    return {"workload": "cu16", "curve": c.tolist(), "iters": [r["iters"] for r in reps],
            "E33": [r["E"][2] for r in reps], "tol": 1e-13}


def curve64():
    from oracle import Oracle
    w = synth.workload("cu64")
    q, rho, _ = synth.make_microstructure(w)
    o = Oracle(w.shape, q, rho)
    reps = [o.increment(Loading(), tol=w.tol, max_iter=2000) for _ in range(3)]
    idx = np.random.default_rng(64).choice(w.voxels, 64, replace=False)
    return {"workload": "cu64", "curve": [r["Sigma"][2] for r in reps],
            "Sigma": [list(r["Sigma"]) for r in reps], "iters": [r["iters"] for r in reps],
            "E": [list(r["E"]) for r in reps], "tol": w.tol, "sample_index": idx.tolist(),
            "sigma_sample": o.field("sigma")[:, idx].tolist(),
            "strain_sample": o.field("strain")[:, idx].tolist(),
            "rho_sample": o.field("rho")[idx].tolist()}


def curve128():
    from oracle import Oracle
    w = synth.workload("cu128")
    q, rho, _ = synth.make_microstructure(w)
    o = Oracle(w.shape, q.reshape(4, -1), rho.reshape(-1))
    r = o.increment(Loading(), tol=w.tol, max_iter=2000)
    idx = np.random.default_rng(128).choice(w.voxels, 256, replace=False)
    return {"workload": "cu128", "increments": 1, "curve": [r["Sigma"][2]], "Sigma": [list(r["Sigma"])],
            "iters": [r["iters"]], "E": [list(r["E"])], "tol": w.tol, "err_c": r["err_c"],
            "err_bc": r["err_bc"], "sample_index": idx.tolist(),
            "sigma_sample": o.field("sigma")[:, idx].tolist(),
            "strain_sample": o.field("strain")[:, idx].tolist(),
            "epsp_sample": o.field("epsp")[:, idx].tolist(),
            "rho_sample": o.field("rho")[idx].tolist()}


if __name__ == "__main__":
    which = sys.argv[1:] or ["adjoint", "curve16"]
    if "adjoint" in which:
        with open(os.path.join(HERE, "adjoint_8cube.json"), "w") as fh:
            json.dump(adjoint_case(), fh, indent=1)
    if "curve16" in which:
        with open(os.path.join(HERE, "curve_16cube.json"), "w") as fh:
            json.dump(curve16(), fh, indent=1)
    if "curve128" in which:
        with open(os.path.join(HERE, "curve_128cube.json"), "w") as fh:
            json.dump(curve128(), fh, indent=1)
    if "curve64" in which:
        with open(os.path.join(HERE, "curve_64cube.json"), "w") as fh:
            json.dump(curve64(), fh, indent=1)
