"""CPU-only checks of the C ABI: the library loads, exports every function that
a header under include/ declares, and validates arguments before touching a
device; the build flags keep packed FP32 off and FMA contraction explicit."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_2511_22468_amd", "libdnb.so")


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(dnb_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_all_headers_are_scanned():
    names = {os.path.basename(h) for h in HEADERS}
    assert {"dnb.h", "dnb_surrogate.h", "dnb_orbitfit.h"} <= names
    fns = declared_functions()
    for must in ("dnb_mlp_forward", "dnb_track_lm", "dnb_simulate_batch", "dnb_mmd_batch"):
        assert must in fns


def test_build_flags():
    from paper_2511_22468_amd import build
    flags = " ".join(build.FLAGS)
    assert "--offload-arch=gfx950" in flags
    assert "-Xclang -target-feature -Xclang -packed-fp32-ops" in flags
    assert "-ffp-contract=off" in flags
    assert set(build.SOURCES) == {os.path.basename(p) for p in
                                  glob.glob(os.path.join(ROOT, "paper_2511_22468_amd", "csrc",
                                                         "*.hip"))}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdnb.so is not built (run python -m paper_2511_22468_amd.build)")
    from paper_2511_22468_amd import _lib
    return _lib.load_library(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dnb_create", "dnb_destroy", "dnb_accelerations", "dnb_step", "dnb_simulate",
                 "dnb_simulate_vjp", "dnb_mmd", "dnb_energy", "dnb_orbit", "dnb_orbit_vjp",
                 "dnb_place_plummer", "dnb_place_plummer_vjp", "dnb_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_size_queries(lib):
    assert b"gfx950" in lib.dnb_version()
    assert lib.dnb_tape_doubles(10, 7, 3) == 3 * (90 + 8) + 30
    assert lib.dnb_tape_doubles(10, 0, 3) == 0
    assert lib.dnb_tape_doubles(10, 7, 0) == -1
    assert lib.dnb_vjp_workspace_doubles(10, 4) == 160 + 2 * (3 * 10 * 5 + 3 * 10 * 4)
    assert lib.dnb_vjp_workspace_doubles(10, 1) == 160
    assert lib.dnb_vjp_workspace_doubles(0, 4) == -1


def test_arguments_rejected_before_any_device_work(lib):
    from paper_2511_22468_amd import _lib
    h = ctypes.c_void_p()
    assert lib.dnb_create(None, 10, 0) == _lib.DNB_ERR_ARG
    assert lib.dnb_create(ctypes.byref(h), 0, 0) == _lib.DNB_ERR_ARG
    assert b"max_n" in lib.dnb_last_error()
    assert lib.dnb_create(ctypes.byref(h), 1 << 27, 0) == _lib.DNB_ERR_ARG
    assert lib.dnb_create(ctypes.byref(h), 10, 7) == _lib.DNB_ERR_ARG
    pot = _lib.dnb_pot(4.3e-6, 1e-3, 1e12, 16.0, 6.5e10, 3.0, 0.28)
    assert lib.dnb_accelerations(None, 10, None, None, ctypes.byref(pot), 1, None, None) == _lib.DNB_ERR_ARG
    assert b"ctx is NULL" in lib.dnb_last_error()
    assert lib.dnb_simulate(None, 10, None, None, None, ctypes.byref(pot), 0.1, 5, 1, None, None) == _lib.DNB_ERR_ARG
    assert lib.dnb_mmd(None, 1, None, 1, None, 0.2, None, None, None) == _lib.DNB_ERR_ARG
    assert lib.dnb_accelerations_rows(None, 10, None, None, ctypes.byref(pot), 1, 0, 5, None,
                                      None) == _lib.DNB_ERR_ARG
    assert lib.dnb_accelerations_vjp(None, 10, None, None, ctypes.byref(pot), 1, None, 0, 5,
                                     None, None, None) == _lib.DNB_ERR_ARG
    table = (ctypes.c_double * 8)(4.3e-6, 1e-3, 1e12, 16.0, 6.5e10, 3.0, 0.28, 0.01)
    assert lib.dnb_simulate_batch(None, 1, 10, None, None, None, table, 5, None,
                                  None) == _lib.DNB_ERR_ARG
    assert lib.dnb_orbit_batch(None, 1, None, table, 5, None, None, None) == _lib.DNB_ERR_ARG
    assert lib.dnb_mmd_batch(None, 1, 10, None, 10, None, 0, 0.2, None, None,
                             None) == _lib.DNB_ERR_ARG
    assert lib.dnb_mmd_batch_targets(None, 1, 10, None, 2, 10, None, 0.2, None,
                                     None) == _lib.DNB_ERR_ARG
    assert lib.dnb_batch_capacity(None, 10) == 0
    model = _lib.dnb_track_model()
    assert lib.dnb_track_chi2(None, ctypes.byref(model), 4, None, 1, None, None, None, None,
                              None) == _lib.DNB_ERR_ARG
    assert lib.dnb_track_lm(None, ctypes.byref(model), 4, None, 1, None, 10, 1e-3, None,
                            None) == _lib.DNB_ERR_ARG
    assert b"ctx is NULL" in lib.dnb_last_error()
    assert lib.dnb_simulate_resume(None, 10, None, 20, 5, 1, None, None, None, ctypes.byref(pot),
                                   0.1, 5, 1, None, None) == _lib.DNB_ERR_ARG
    first = ctypes.c_int64(7)
    assert lib.dnb_check_state(None, 10, None, None, None, ctypes.byref(first),
                               None) == _lib.DNB_ERR_ARG
    assert first.value == 7
    assert lib.dnb_set_checks(None, 1) == _lib.DNB_ERR_ARG
    assert b"ctx is NULL" in lib.dnb_last_error()
    lib.dnb_destroy(None)


def test_binding_refuses_to_run_without_the_library(tmp_path):
    from paper_2511_22468_amd import _lib
    with pytest.raises(ImportError):
        _lib.load_library(str(tmp_path / "missing.so"))
