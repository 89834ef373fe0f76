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
    assert lib.gps_polarization_charge_noalloc(None, None, None, None, None) == \
        gps.GPS_E_INVALID
    assert lib.gps_plan_device_bytes(None) == 0
    lib.gps_plan_destroy(None)


def test_footprint_host_side(lib):
    tb, b, t = gps.plan_footprint((96, 96, 96), "free", "mixed")
    tb64, b64, _ = gps.plan_footprint((96, 96, 96), "free", "fp64")
    tbn, bnl, tnl = gps.plan_footprint((96, 96, 96), "free", "mixed", nonlinear_pb=True)
    n = 96 ** 3
    assert bnl - b == 4 * n                      # FP32 ionic-charge field
    assert tnl == t == 192 * 192 * 97 * 16       # FP64 padded half spectrum while planning
    assert tb == tbn == tb64                     # tables do not depend on the precision
    assert tb > 97 ** 3 * 12                     # FP64 + FP32 folded Green table
    assert b64 > b
    # the FP32 work buffer (96 x 192 x 97 complex) and 6 FP32 vectors dominate
    assert b > 96 * 192 * 97 * 8 + 6 * 4 * n
    tbp, bp, tp = gps.plan_footprint((32, 32, 32), "periodic", "mixed")
    assert tp == 0 and bp > 0 and tbp > 0
    # refinement: sigma, s, q and G s in FP64 and an FP64 work buffer; never periodic
    _, br, _ = gps.plan_footprint((96, 96, 96), "free", "mixed", refine=True)
    assert br - b == 4 * 8 * n + 96 * 192 * 97 * 16
    assert gps.plan_footprint((32, 32, 32), "periodic", "mixed", refine=True)[1] == bp
    with pytest.raises(gps.GPSError):
        gps.plan_footprint((1, 8, 8), "free")


def test_server_argument_checks_need_no_device(lib):
    t = ctypes.c_longlong()
    assert lib.gps_server_create(None, None) == gps.GPS_E_INVALID
    bad = gps.gps_server_options(0, 0, 1, 16, 100, 4)       # max_active 0
    h = ctypes.c_void_p()
    assert lib.gps_server_create(ctypes.byref(bad), ctypes.byref(h)) == gps.GPS_E_INVALID
    bad = gps.gps_server_options(0, 4, 1, 16, 100, 9)       # batch_slots beyond 8
    assert lib.gps_server_create(ctypes.byref(bad), ctypes.byref(h)) == gps.GPS_E_INVALID
    assert lib.gps_server_submit(None, None, ctypes.byref(t)) == gps.GPS_E_INVALID
    assert lib.gps_server_poll(None, 1, None) == gps.GPS_E_INVALID
    assert lib.gps_server_wait(None, 1, None) == gps.GPS_E_INVALID
    assert lib.gps_server_get_stats(None, None) == gps.GPS_E_INVALID
    lib.gps_server_destroy(None)
    assert lib.gps_plan_release_buffers(None) == gps.GPS_E_INVALID
    assert lib.gps_status_string(8) == b"pending"
