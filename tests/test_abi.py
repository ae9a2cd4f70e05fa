"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/fem.h declares, and rejects invalid arguments before touching a
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    text = open(os.path.join(ROOT, "include", "fem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fem.LIB_PATH):
        from paper_2103_16747_amd import build
        build.build()
    return fem.load()


def test_exports_every_declared_entry_point(lib):
    names = declared_entry_points()
    assert len(names) >= 14
    assert set(names) == set(fem.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


def test_library_has_gfx950_code_object():
    blob = open(fem.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_status_strings(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8):
        assert lib.fem_status_string(code).decode() not in ("", "unknown status")
    assert lib.fem_status_string(-99).decode() == "unknown status"


def test_default_params(lib):
    p64 = fem.fem_default_params(fem.FEM_PREC_FP64)
    p32 = fem.fem_default_params(fem.FEM_PREC_FP32)
    assert p64.newton_rtol == 1e-8 and p64.precond == 1 and p64.contact_hessian == 1
    assert p32.newton_rtol > p64.newton_rtol
    assert p64.newton_floor_rtol > p64.newton_rtol and p32.newton_floor_rtol > p32.newton_rtol
    assert p64.cg_eta_power == 1.0 and p32.cg_eta_power == 0.75


def _create(lib, X, T, F):
    h = C.c_void_p()
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.int32)
    F = np.ascontiguousarray(F, dtype=np.uint8)
    rc = lib.fem_create_mesh(X.ctypes.data_as(C.POINTER(C.c_double)), X.shape[0],
                             T.ctypes.data_as(C.POINTER(C.c_int32)), T.shape[0],
                             F.ctypes.data_as(C.POINTER(C.c_uint8)), None, C.byref(h))
    return rc, h


def test_create_rejects_bad_input_before_device(lib):
    m = W.block_mesh((1, 1, 1), (1e-3, 1e-3, 1e-3))
    bad_index = m.tets.copy()
    bad_index[0, 0] = m.n
    assert _create(lib, m.X, bad_index, m.fixed)[0] == fem.FEM_E_INVALID
    assert "range" in lib.fem_last_error().decode()
    neg = m.tets.copy()
    neg[0, 0] = -1
    assert _create(lib, m.X, neg, m.fixed)[0] == fem.FEM_E_INVALID
    nanX = m.X.copy()
    nanX[3, 1] = np.nan
    assert _create(lib, nanX, m.tets, m.fixed)[0] == fem.FEM_E_INVALID
    assert _create(lib, m.X[:0], m.tets[:0], m.fixed[:0])[0] == fem.FEM_E_INVALID
    h = C.c_void_p()
    assert lib.fem_create_mesh(None, 3, None, 1, None, None, C.byref(h)) == fem.FEM_E_INVALID
    assert lib.fem_create_mesh(None, 3, None, 1, None, None, None) == fem.FEM_E_INVALID


def test_calls_on_null_handle_fail_cleanly(lib):
    assert lib.fem_set_material(None, 1.0, 0.3, 0.0) == fem.FEM_E_INVALID
    assert lib.fem_step(None, None, None) == fem.FEM_E_INVALID
    lib.fem_destroy_mesh(None)


def test_oracle_is_separate_library(oracle_lib):
    # The oracle is its own shared object and the device library does not link it.
    blob = open(fem.LIB_PATH, "rb").read()
    assert b"orc_" not in blob
    assert os.path.exists(oracle_lib.LIB_PATH)
