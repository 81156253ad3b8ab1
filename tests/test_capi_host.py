"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function include/naj.h declares, and the option defaults match the header."""
import ctypes
import os

import pytest

from paper_2407_03272_amd import naj


def test_library_exports_every_declared_symbol():
    lib = naj.load()
    names = naj.header_functions()
    assert len(names) >= 10
    missing = [f for f in names if not hasattr(lib, f)]
    assert not missing, missing
    # the binding declares signatures for exactly the header's functions
    assert sorted(naj._SIGS) == names


def test_opts_defaults_and_struct_layout():
    o = naj.default_opts()
    assert o.tol == 1e-8 and o.max_iter == 20000 and o.restart == 1 and o.k0 == 2
    assert o.confirm_gap == 8 and o.precision == naj.NAJ_FP64 and o.inner_stall == 200
    assert o.stop == naj.NAJ_STOP_RELRES and o.fstar == 0.0
    assert ctypes.sizeof(naj.NajOpts) == 64
    assert ctypes.sizeof(naj.NajResult) == 56


def test_version_and_error_string():
    lib = naj.load()
    assert lib.naj_version().decode().startswith("naj")
    assert lib.naj_last_error() is not None


def test_invalid_arguments_rejected_before_device_work():
    lib = naj.load()
    h = ctypes.c_void_p()
    assert lib.naj_create_system(0, 0, None, None, None, None, None, ctypes.byref(h)) == naj.NAJ_EINVAL
    assert b"n must be" in lib.naj_last_error()
    assert lib.naj_create_system(10, -1, None, None, None, None, None, ctypes.byref(h)) == naj.NAJ_EINVAL
    assert lib.naj_create_system(10, 5, None, None, None, None, None, None) == naj.NAJ_EINVAL
    res = naj.NajResult()
    assert lib.naj_solve(None, None, None, None, None, ctypes.byref(res), None, 0, None, 0, None, 0, None) \
        == naj.NAJ_EINVAL


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="build the HIP library"):
        naj._lib_backup = naj._lib
        try:
            naj._lib = None
            naj.load(str(tmp_path / "nope.so"))
        finally:
            naj._lib = naj._lib_backup
