"""The C-ABI library loads, exports every symbol include/dr.h declares, and
rejects bad arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dr.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:dr_status|const char\*)\s+(dr_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2201_13309_amd import dr
    return dr.load()


def test_header_parses():
    syms = declared_symbols()
    assert "dr_reconstruct" in syms and "dr_submit" in syms and len(syms) >= 18


def test_every_declared_symbol_is_exported(lib):
    from paper_2201_13309_amd import dr
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(declared_symbols()) == set(dr.ABI_SYMBOLS)


def test_null_arguments_rejected_without_device(lib):
    from paper_2201_13309_amd import dr
    assert lib.dr_reconstruct(None, None, 1, None, None, None) == dr.DR_E_INVAL
    assert "NULL" in dr.dr_last_error()
    assert lib.dr_reconstruct_f64(None, None, None, None, None) == dr.DR_E_INVAL
    assert lib.dr_reconstruct_noalloc(None, None, None, None, None) == dr.DR_E_INVAL
    assert lib.dr_geometry_init(None, None, None, None, None) == dr.DR_E_INVAL
    assert lib.dr_geometry_free(None) == dr.DR_E_INVAL
    assert lib.dr_ctx_destroy(None) == dr.DR_E_INVAL
    assert lib.dr_batch_create(None, 0, None, 0, None) == dr.DR_E_INVAL
    assert lib.dr_batch_run(None, None) == dr.DR_E_INVAL
    t = ctypes.c_uint64()
    assert lib.dr_submit(None, None, None, 0, None, None, ctypes.byref(t)) == dr.DR_E_INVAL
    assert lib.dr_poll(None, 1) == dr.DR_E_INVAL
    assert lib.dr_ctx_create(0, 0, None) == dr.DR_E_INVAL
    assert lib.dr_debug_plan(None, None, 0, 0, None, None) == dr.DR_E_INVAL
    assert lib.dr_pixel_activity(None, None, None, None) == dr.DR_E_INVAL
    assert lib.dr_select_top(None, None, 0, None) == dr.DR_E_INVAL
    assert lib.dr_list_create(None, None, 0, 0, None) == dr.DR_E_INVAL
    assert lib.dr_list_free(None) == dr.DR_E_INVAL
    assert lib.dr_reconstruct_list(None, None, 0, 1, None, None, None) == dr.DR_E_INVAL
    assert lib.dr_reconstruct_list_f64(None, None, 0, None, None, None) == dr.DR_E_INVAL
    assert lib.dr_geometry_path(None, None) == dr.DR_E_INVAL
    assert lib.dr_geometry_position_margin(None, None, None) == dr.DR_E_INVAL
    assert lib.dr_geometry_set_step_weights(None, None) == dr.DR_E_INVAL


def test_ctx_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2201_13309_amd import dr
    h = ctypes.c_void_p()
    rc = lib.dr_ctx_create(0, 0, ctypes.byref(h))
    assert rc in (dr.DR_E_DEVICE, dr.DR_E_INVAL) and not h.value
