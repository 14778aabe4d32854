"""CPU oracle for the FFT-EVP fixed-point solve — TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 implementation (numpy) of what the GPU path computes,
written from the paper's statement of the method (Sec. 2.1, Eq. 1-2: implicit
Euler Hooke law, plastic rate as a sum over slip systems, spectral solution of
equilibrium, augmented-Lagrangian treatment of the nonlinear local equations)
and from the readings recorded for the points the paper leaves open.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package. The product path (the HIP library and its Python
binding) never imports, links or calls it, and the two share no code: the
oracle works in the sample frame with full fourth-order tensors, builds the
Green operator through the acoustic tensor, uses numpy's FFT and solves the
local problem with dense linear algebra, while the GPU path uses its own
formulations of each step.

Parity pins (tests under ``tests/`` marked ``not gpu``) tie every function
here to values fixed independently of the oracle: closed-form elastic moduli,
the analytic plastic steady state and Kocks-Mecking saturation law of a
single crystal, laminate solutions, Voigt/Reuss bounds, Green-operator
identities, brute-force DFTs and convexity of the local problem.
"""
from .solve import Oracle, Flow, Loading, default_c0, run_path, stress_curve, fd_gradient, curve_loss, CU  # noqa: F401
