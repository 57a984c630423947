"""CPU checks of the C ABI library: it loads, exports every entry point declared in
include/shearseg.h, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1112_1805_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shearseg.h")

pytestmark = pytest.mark.skipif(not os.path.exists(pkg.LIB_PATH), reason="library not built")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(shs_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for name in ["shs_plan_create", "shs_plan_destroy", "shs_workspace_bytes", "shs_state_bytes",
                 "shs_num_filters", "shs_filters", "shs_datacost", "shs_shearlet_forward",
                 "shs_shearlet_adjoint", "shs_shearlet_denoise", "shs_solve", "shs_solve_pd", "shs_solve_tv", "shs_energy", "shs_status_str", "shs_last_error",
                 "shs_batch_create", "shs_batch_destroy", "shs_batch_workspace_bytes", "shs_solve_batch",
                 "shs_profile_begin", "shs_profile_end"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(pkg.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(L, s)]
    assert not missing, missing
    assert set(declared_symbols()) == set(pkg._SIGS)


def test_pure_host_entry_points():
    L = pkg.lib()
    assert [L.shs_num_filters(J) for J in (1, 2, 3, 4)] == [5, 13, 29, 61]
    assert L.shs_num_filters(0) == -1
    assert L.shs_workspace_bytes(None) == 0 and L.shs_state_bytes(None) == 0
    assert L.shs_status_str(pkg.SHS_E_WORKSPACE) == b"workspace too small or missing"
    assert L.shs_plan_destroy(None) == pkg.SHS_OK


@pytest.mark.parametrize("shape,code", [
    ((100, 1, 3, 2, 0), pkg.SHS_E_UNSUPPORTED),   # size not supported
    ((128, 1, 0, 2, 0), pkg.SHS_E_INVALID),       # q < 1
    ((128, 1, 9, 2, 0), pkg.SHS_E_INVALID),       # q > 8
    ((128, 5, 3, 2, 0), pkg.SHS_E_INVALID),       # channels > 4
    ((128, 1, 3, 0, 0), pkg.SHS_E_INVALID),       # J < 1
    ((128, 1, 3, 5, 0), pkg.SHS_E_INVALID),       # 4^J > 2N
    ((128, 1, 3, 2, 7), pkg.SHS_E_INVALID),       # bad storage type
])
def test_plan_validation(shape, code):
    L = pkg.lib()
    h = ctypes.c_void_p()
    st = L.shs_plan_create(ctypes.byref(pkg.ShsShape(*shape)), 0, ctypes.byref(h))
    assert st == code and not h.value
    assert len(L.shs_last_error()) > 0


def test_batch_validation_without_device():
    L = pkg.lib()
    h = ctypes.c_void_p()
    bad = (pkg.ShsShape * 2)(pkg.ShsShape(128, 1, 3, 2, 0), pkg.ShsShape(100, 1, 3, 2, 0))
    assert L.shs_batch_create(0, bad, 0, ctypes.byref(h)) == pkg.SHS_E_INVALID
    assert L.shs_batch_create(2, None, 0, ctypes.byref(h)) == pkg.SHS_E_INVALID
    assert L.shs_batch_workspace_bytes(None) == 0 and L.shs_batch_destroy(None) == pkg.SHS_OK
    assert L.shs_solve_batch(None, None, None, None, 0, None, None, None, None) == pkg.SHS_E_INVALID


def test_null_arguments():
    L = pkg.lib()
    assert L.shs_plan_create(None, 0, None) == pkg.SHS_E_INVALID
    assert L.shs_solve(None, None, None, None, 0, None, None, None, None, None) == pkg.SHS_E_INVALID
    assert L.shs_shearlet_forward(None, 1, None, None, None, 0, None) == pkg.SHS_E_INVALID
    assert L.shs_shearlet_denoise(None, 1, None, 0, None, None, None, 0, None) == pkg.SHS_E_INVALID
    assert L.shs_solve_pd(None, None, None, None, 0, None, None, None, None, None) == pkg.SHS_E_INVALID
    assert L.shs_solve_tv(None, None, None, None, 0, None, None, None, None, None) == pkg.SHS_E_INVALID
