"""C-ABI contract checks that need no GPU: the library loads, exports every
entry point declared in include/fpde.h, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1811_03339_amd as F

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fpde.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpde_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared()
    assert len(names) >= 13
    L = F._lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(F.EXPORTS)


def test_status_strings():
    L = F._lib()
    for code in F.STATUS:
        s = L.fpde_status_string(code)
        assert s and s != b"unknown status"
    assert L.fpde_status_string(12345) == b"unknown status"


def test_mesh_create_rejects_bad_input_without_device():
    L = F._lib()
    h = ctypes.c_void_p()
    xyz = np.zeros((4, 3))
    tet = np.array([[0, 1, 2, 7]], dtype=np.int32)  # vertex id out of range
    st = L.fpde_mesh_create(xyz.ctypes.data_as(ctypes.c_void_p), 4, tet.ctypes.data_as(ctypes.c_void_p), 1,
                            None, ctypes.byref(h))
    assert st == -1 and not h.value
    st = L.fpde_mesh_create(None, 4, None, 1, None, ctypes.byref(h))
    assert st == -1
    bad = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, np.nan]])
    tet = np.array([[0, 1, 2, 3]], dtype=np.int32)
    st = L.fpde_mesh_create(bad.ctypes.data_as(ctypes.c_void_p), 4, tet.ctypes.data_as(ctypes.c_void_p), 1,
                            None, ctypes.byref(h))
    assert st == -1


def test_calls_on_null_handle_are_rejected():
    L = F._lib()
    p = F.params(1.5)
    assert L.fpde_assemble(None, ctypes.byref(p), None, 0, None, None, None) == -1
    assert L.fpde_solve(None, ctypes.byref(p), None, 0, None, None, None, None) == -1
    assert L.fpde_plan(None, 4, 0, None) == -1
    assert L.fpde_mesh_info(None, None, None, None) == -1


def test_params_layout_matches_header():
    # double alpha; double K[3]; int quad_points, precision, source, max_steps;
    # double ir_tol; int ir_max_iter, deterministic (in the former tail padding)
    assert ctypes.sizeof(F.fpde_params) == 8 + 24 + 16 + 8 + 8
    assert F.fpde_params.ir_tol.offset == 48
    assert F.fpde_params.deterministic.offset == 60
    assert ctypes.sizeof(F.fpde_solve_info) == 24


def test_div_params_layout_matches_header():
    # double beta[3]; int quad_points, coef, source; double radius; int max_steps
    assert F.fpde_div_params.radius.offset == 40
    assert ctypes.sizeof(F.fpde_div_params) == 56


def test_div_and_lu_calls_reject_bad_arguments_without_device():
    L = F._lib()
    p = F.div_params((0.8, 0.8, 0.8))
    assert L.fpde_div_assemble(None, ctypes.byref(p), None, None, 0, None, None, None) == -1
    assert L.fpde_lu_factor(None, None, 0, None, None) == -1
    assert L.fpde_lu_solve(None, None, 0, None, None, None) == -1


def test_params2d_layout_and_null_handles():
    # double alpha; double K[2]; int quad_points, source, max_steps
    assert F.fpde_params2d.quad_points.offset == 24
    assert ctypes.sizeof(F.fpde_params2d) == 40
    L = F._lib()
    p = F.params2d(1.5)
    assert L.fpde_assemble2d(None, ctypes.byref(p), None, 0, None, None, None) == -1
    assert L.fpde_mesh2d_info(None, None, None, None) == -1
    h = ctypes.c_void_p()
    xy = np.zeros((3, 2))
    tri = np.array([[0, 1, 5]], dtype=np.int32)
    assert L.fpde_mesh2d_create(xy.ctypes.data_as(ctypes.c_void_p), 3, tri.ctypes.data_as(ctypes.c_void_p), 1,
                                None, ctypes.byref(h)) == -1


def test_fracsolve_refuses_sources_that_depend_on_alpha_or_K():
    import torch
    a = torch.tensor(1.5, dtype=torch.float64, requires_grad=True)
    k = torch.ones(3, dtype=torch.float64, requires_grad=True)
    # rejected before any device work (the mesh is never touched)
    with pytest.raises(ValueError):
        F.FracSolve.apply(a, k, None, 4, F.FPDE_FP64, F.FPDE_SRC_CUBE_MMS)
