"""The C-ABI library loads and exports every symbol include/gps.h declares;
host-side argument checks answer without a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_1509_00680_amd import gps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "gps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gps_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gps.LIB_PATH):
        from paper_1509_00680_amd import build
        build.build()
    return gps.load()


def test_every_declared_symbol_exported(lib):
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(gps.EXPORTED) == names


def test_status_strings(lib):
    assert lib.gps_status_string(0) == b"ok"
    assert lib.gps_status_string(7) == b"unsupported size"
    assert lib.gps_status_string(99) == b"unknown status"


def test_plan_argument_checks_need_no_device(lib):
    out = ctypes.c_void_p()
    assert lib.gps_plan_create(1, 8, 8, 0.5, 0, ctypes.byref(out)) == gps.GPS_E_INVALID
    assert lib.gps_plan_create(8, 8, 8, -1.0, 0, ctypes.byref(out)) == gps.GPS_E_INVALID
    assert lib.gps_plan_create(8, 8, 8, 0.5, 9, ctypes.byref(out)) == gps.GPS_E_INVALID
    assert lib.gps_plan_create(11, 8, 8, 0.5, 0, ctypes.byref(out)) == gps.GPS_E_UNSUPPORTED
    assert lib.gps_plan_create(8, 8, 600, 0.5, 0, ctypes.byref(out)) == gps.GPS_E_UNSUPPORTED
    assert lib.gps_plan_create(8, 8, 8, 0.5, 0, None) == gps.GPS_E_INVALID
    assert not out.value


def test_null_plan_rejected(lib):
    o = gps.gps_options(0, 16, 100, 8, None)
    assert lib.gps_plan_set_options(None, ctypes.byref(o)) == gps.GPS_E_INVALID
    assert lib.gps_solve_generalized(None, None, None, None, 1e-6) == gps.GPS_E_INVALID
    assert lib.gps_plan_set_timing(None, 1) == gps.GPS_E_INVALID
    assert lib.gps_last_info(None, None) == gps.GPS_E_INVALID
    assert lib.gps_plan_device_bytes(None) == 0
    lib.gps_plan_destroy(None)
