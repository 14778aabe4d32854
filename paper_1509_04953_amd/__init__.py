"""MI355X-native FFT-EVP fixed-point solve (small-strain crystal plasticity).

The solve runs in ``libfftevp.so`` (hand-written HIP for gfx950, C ABI in
``include/fftevp.h``); this package is its thin Python binding.
"""
from .fftevp import (Solver, PhaseField, Material, MaRoters, Load, Opts, Report, FftevpError, library,  # noqa: F401
                     OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENONFINITE, ELOCAL, ESTATE)
