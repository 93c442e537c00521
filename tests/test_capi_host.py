"""C ABI checks that run without a GPU: exports and argument validation.

Every function declared in include/thx.h must be exported by libthx.so, and
the calls whose arguments are invalid must return THX_INVALID_ARGUMENT (or
THX_UNSUPPORTED) before touching the device.
"""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "thx.h")
LIB = os.path.join(ROOT, "paper_1604_07486_amd", "libthx.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(thx_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libthx.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_entry_points():
    names = _declared()
    for must in ["thx_plan_create", "thx_execute", "thx_plan_destroy", "thx_leg2cheb", "thx_cheb2leg",
                 "thx_ultra2ultra", "thx_lag2lag", "thx_lambda_table", "thx_status_string"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (thx_[a-z0-9_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        getattr(lib, n)  # resolvable through the dynamic loader


def test_status_strings(lib):
    lib.thx_status_string.restype = ctypes.c_char_p
    for code, name in enumerate(["THX_OK", "THX_INVALID_ARGUMENT", "THX_UNSUPPORTED", "THX_TOL_NOT_REACHED",
                                 "THX_OUT_OF_MEMORY", "THX_HIP_ERROR", "THX_WORKSPACE_TOO_LARGE"]):
        assert lib.thx_status_string(code).decode() == name


def _create(lib, kind, params, degree, tol, prec=0, flags=0):
    h = ctypes.c_void_p()
    arr = (ctypes.c_double * max(1, len(params)))(*params)
    lib.thx_plan_create.restype = ctypes.c_int
    lib.thx_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_uint32,
                                    ctypes.c_void_p]
    st = lib.thx_plan_create(ctypes.byref(h), kind, arr, len(params), degree, tol, prec, flags, None)
    return st, h


@pytest.mark.parametrize("kind,params,degree,tol,prec,expect", [
    (0, (), -1, 1e-15, 0, 1),          # negative degree
    (0, (), 10, 0.0, 0, 1),            # tol must be in (0, 1)
    (0, (), 10, 1.5, 0, 1),
    (0, (), 10, float("nan"), 0, 1),
    (0, (), 10, 1e-15, 7, 1),          # unknown precision
    (0, (), 10, 1e-15, 3, 1),          # one past THX_FP64_TAIL32
    (2, (), 10, 1e-15, 0, 1),          # ultra2ultra needs two parameters
    (2, (-0.5, 0.5), 10, 1e-15, 0, 1), # lambda must be > 0
    (4, (-1.5, 0.0), 10, 1e-15, 0, 1), # Laguerre parameter must be > -1
    (9, (), 10, 1e-15, 0, 2),          # unknown kind
])
def test_plan_create_rejects(lib, kind, params, degree, tol, prec, expect):
    st, h = _create(lib, kind, params, degree, tol, prec)
    assert st == expect and not h.value


def test_null_out_pointer(lib):
    lib.thx_plan_create.restype = ctypes.c_int
    assert lib.thx_plan_create(None, 0, None, 0, ctypes.c_int64(10), ctypes.c_double(1e-15), 0,
                               ctypes.c_uint32(0), None) == 1


def test_execute_rejects_null_plan(lib):
    lib.thx_execute.restype = ctypes.c_int
    lib.thx_execute.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64] * 3 + [ctypes.c_void_p]
    assert lib.thx_execute(None, None, None, 10, 1, 11, None) == 1


def test_introspection_null_plan(lib):
    lib.thx_plan_rank.restype = ctypes.c_int32
    lib.thx_plan_path.restype = ctypes.c_int32
    lib.thx_plan_fft_length.restype = ctypes.c_int64
    lib.thx_plan_destroy.restype = ctypes.c_int
    assert lib.thx_plan_rank(None) == -1
    assert lib.thx_plan_path(None) == -1
    assert lib.thx_plan_fft_length(None) == -1
    assert lib.thx_plan_destroy(None) == 0
    lib.thx_plan_autotune.restype = ctypes.c_int
    lib.thx_plan_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    assert lib.thx_plan_autotune(None, 4, None) == 1          # THX_INVALID_ARGUMENT
    lib.thx_plan_fft_geometry.restype = ctypes.c_int
    lib.thx_plan_fft_geometry.argtypes = [ctypes.c_void_p] * 4
    assert lib.thx_plan_fft_geometry(None, None, None, None) == 1
    lib.thx_plan_launch_shape.restype = ctypes.c_int
    lib.thx_plan_launch_shape.argtypes = [ctypes.c_void_p] * 3
    assert lib.thx_plan_launch_shape(None, None, None) == 1
    lib.thx_plan_lds_radix.restype = ctypes.c_int32
    lib.thx_plan_lds_radix.argtypes = [ctypes.c_void_p]
    assert lib.thx_plan_lds_radix(None) == -1
    lib.thx_plan_p1_blocks.restype = ctypes.c_int32
    lib.thx_plan_p1_blocks.argtypes = [ctypes.c_void_p]
    assert lib.thx_plan_p1_blocks(None) == -1
    lib.thx_plan_fused_columns.restype = ctypes.c_int32
    lib.thx_plan_fused_columns.argtypes = [ctypes.c_void_p]
    assert lib.thx_plan_fused_columns(None) == -1
    lib.thx_plan_tail_slots.restype = ctypes.c_int32
    lib.thx_plan_tail_slots.argtypes = [ctypes.c_void_p]
    assert lib.thx_plan_tail_slots(None) == -1
    lib.thx_plan_enable_timing.restype = ctypes.c_int
    lib.thx_plan_enable_timing.argtypes = [ctypes.c_void_p, ctypes.c_uint32]
    assert lib.thx_plan_enable_timing(None, 0xFFFFFFFF) == 1
    lib.thx_plan_partial_groups.restype = ctypes.c_int32
    lib.thx_plan_partial_groups.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    assert lib.thx_plan_partial_groups(None, 1) == 0


def test_table_rejects_negative_count(lib):
    lib.thx_lambda_table.restype = ctypes.c_int
    lib.thx_lambda_table.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p]
    assert lib.thx_lambda_table(None, -1, 0.0, None) == 1
    assert lib.thx_lambda_table(None, 5, 0.0, None) == 1


@pytest.mark.parametrize("kind,params", [(3, (0.5, 0.5, 0.5)), (5, (-1.5, 0.0)), (6, (0.0,))])
def test_jacobi_bad_parameters(lib, kind, params):
    st, h = _create(lib, kind, params, 50, 1e-15)
    assert st == 1 and not h.value


def test_boundary_calls_declared():
    # the paper's commands (Sec. 1, 5.1-5.4) and the variable-length execution
    names = _declared()
    for must in ["thx_jac2jac", "thx_jac2cheb", "thx_cheb2jac", "thx_execute_varlen", "thx_batch_create",
                 "thx_plan_achieved_tol", "thx_last_hip_error"]:
        assert must in names


@pytest.mark.parametrize("fname,args", [
    ("thx_jac2jac", (0.5, 0.5, 0.5, -1.5)),     # parameters must be > -1
    ("thx_jac2jac", (-1.0, 0.5, 0.5, 0.5)),
    ("thx_jac2cheb", (-1.5, 0.0)),
    ("thx_cheb2jac", (0.0, -2.0)),
])
def test_jacobi_oneshots_reject_parameters(lib, fname, args):
    f = getattr(lib, fname)
    f.restype = ctypes.c_int
    f.argtypes = ([ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_double] * (len(args) + 1)
                  + [ctypes.c_int, ctypes.c_void_p])
    assert f(None, None, 10, 1, *args, 1e-15, 0, None) == 1


def test_oneshot_rejects_negative_degree(lib):
    lib.thx_jac2cheb.restype = ctypes.c_int
    lib.thx_jac2cheb.argtypes = ([ctypes.c_void_p] * 2 + [ctypes.c_int64] * 2 + [ctypes.c_double] * 3
                                 + [ctypes.c_int, ctypes.c_void_p])
    assert lib.thx_jac2cheb(None, None, -1, 1, 0.5, -0.25, 1e-15, 0, None) == 1


def test_varlen_rejects_bad_arguments(lib):
    f = lib.thx_execute_varlen
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int64] * 2 + [ctypes.c_void_p] * 2
    assert f(None, None, None, None, 3, 10, None, None) == 1     # null plan
    assert f(None, None, None, None, 0, 0, None, None) == 1      # null plan even with nothing to do


def test_last_hip_error_starts_clear(lib):
    lib.thx_last_hip_error.restype = ctypes.c_int
    assert lib.thx_last_hip_error() == 0


def test_noalloc_rejects_null_plan_and_states_scratch(lib):
    lib.thx_execute_noalloc.restype = ctypes.c_int
    lib.thx_execute_noalloc.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64] * 3 + [ctypes.c_void_p]
    assert lib.thx_execute_noalloc(None, None, None, 10, 1, 11, None) == 1
    lib.thx_noalloc_scratch_bytes.restype = ctypes.c_int64
    assert lib.thx_noalloc_scratch_bytes() == 512 << 20
