"""The C ABI: the library loads and exports every declared symbol; argument
checks that return before any device work behave as documented. No GPU."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADERS = sorted((ROOT / "include").glob("*.h"))
LIB = ROOT / "paper_1509_04953_amd" / "libfftevp.so"


@pytest.fixture(scope="module")
def lib():
    if not LIB.exists():
        pytest.fail(f"{LIB} not built: run `python -m paper_1509_04953_amd.build`")
    from paper_1509_04953_amd import library
    return library()


def declared():
    text = "".join(h.read_text() for h in HEADERS)
    return sorted(set(re.findall(r"\b(fftevp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 24 and "fftevp_pf_steps" in names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.fftevp_status_string(s)
    assert lib.fftevp_status_string(1) == b"not converged"


@pytest.mark.parametrize("dims", [(0, 16, 16), (12, 16, 16), (16, 1024, 16), (16, 16, 4), (16, 16, -8)])
def test_create_rejects_bad_grids(lib, dims):
    h = C.c_void_p()
    assert lib.fftevp_create(*dims, 0, None, C.byref(h)) == -1
    assert not h.value


def test_create_rejects_bad_precision_and_null_out(lib):
    h = C.c_void_p()
    assert lib.fftevp_create(16, 16, 16, 7, None, C.byref(h)) == -1
    assert lib.fftevp_create(16, 16, 16, 0, None, None) == -1


def test_null_context_calls(lib):
    assert lib.fftevp_step(None, None, None) == -1
    assert lib.fftevp_destroy(None) == -1
    assert lib.fftevp_set_material(None, None, None) == -1
    assert lib.fftevp_set_loading(None, None) == -1
    assert lib.fftevp_get_field(None, 0, None) == -1
    assert lib.fftevp_state_bytes(None) == 0
    assert lib.fftevp_set_profiling(None, 1) == -1
    assert lib.fftevp_last_error(None) == b"null context"


@pytest.mark.parametrize("args", [(0, 4, 4, 6, 1e-5, 0), (4, 4, 4, 0, 1e-5, 0), (4, 4, 4, 7, 1e-5, 0),
                                  (4, 4, 4, 6, -1.0, 0), (4, 4, 4, 6, 1.0, 0), (4, 4, 4, 6, 1e-5, 3),
                                  (1024, 1024, 512, 6, 1e-5, 0)])
def test_pf_create_rejects_bad_arguments(lib, args):
    h = C.c_void_p()
    assert lib.fftevp_pf_create(*args, None, C.byref(h)) == -1
    assert not h.value


def test_pf_null_context_calls(lib):
    assert lib.fftevp_pf_destroy(None) == -1
    assert lib.fftevp_pf_steps(None, 1) == -1
    assert lib.fftevp_pf_refine(None, None, None) == -1
    assert lib.fftevp_pf_export(None, None, None) == -1
    assert lib.fftevp_pf_grains(None, None, None) == -1
    assert lib.fftevp_pf_import(None, None, None, 1, None) == -1
    assert lib.fftevp_pf_last_error(None) == b"null context"


def test_pf_step_count_on_the_host(lib):
    """floor(dt / (0.225 omega / M)) (Sec. 2.4), -1 for bad arguments."""
    lib.fftevp_pf_step_count.restype = C.c_int
    lib.fftevp_pf_step_count.argtypes = [C.c_double] * 3
    assert lib.fftevp_pf_step_count(1.0, 0.625, 145e-6) == 0          # one step lasts ~970 s
    assert lib.fftevp_pf_step_count(1000.0, 0.625, 145e-6) == 1
    assert lib.fftevp_pf_step_count(9.0, 1.0, 1.0) == 40              # 9 / 0.225
    assert lib.fftevp_pf_step_count(0.0, 1.0, 1.0) == -1
    assert lib.fftevp_pf_step_count(1.0, float("nan"), 1.0) == -1
    assert lib.fftevp_pf_step_count(1e300, 1.0, 1.0) == -1            # beyond int range
    n = C.c_int()
    assert lib.fftevp_pf_dims(None, C.byref(n), C.byref(n), C.byref(n)) == -1
    assert lib.fftevp_drx_grow(None, None, None, 1, None, None) == -1
