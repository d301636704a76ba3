"""The C ABI: the library loads, exports every entry point that include/cdm.h
declares, and rejects invalid descriptors before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cdm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(cdm_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1902_08653_amd import cdm
    if not os.path.exists(cdm.LIB_PATH):
        from paper_1902_08653_amd import build
        build.build()
    return cdm.lib()


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ["cdm_create", "cdm_solve", "cdm_destroy", "cdm_create_batched", "cdm_solve_batched",
              "cdm_residual", "cdm_status_string"]:
        assert f in fns


def test_every_declared_symbol_is_exported(lib):
    from paper_1902_08653_amd import cdm
    fns = declared_functions()
    missing = [f for f in fns if not hasattr(lib, f)]
    assert not missing, missing
    assert sorted(cdm.EXPORTS) == fns


def test_version_and_status_strings(lib):
    assert lib.cdm_version() == 2
    assert lib.cdm_status_string(0) == b"ok"
    assert b"infeasible" in lib.cdm_status_string(-6)
    assert lib.cdm_status_string(12345) == b"unknown status"


def _desc(**kw):
    from paper_1902_08653_amd import cdm
    d = dict(problem=0, precision=0, layout=0, engine=0, B=64, U=16, C=1, T_max=3, tol=0.0, nnz=0,
             panel=0, flags=0)
    d.update(kw)
    return cdm.Desc(**d)


@pytest.mark.parametrize("kw,status", [
    (dict(T_max=0), -1),
    (dict(tol=-1.0), -1),
    (dict(tol=float("nan")), -1),
    (dict(engine=7), -1),
    (dict(precision=9), -3),
    (dict(problem=5), -3),
    (dict(B=0), -2),
    (dict(U=0), -2),
    (dict(B=65, C=2), -2),
    (dict(problem=1, B=32, U=16, C=4), -6),      # downlink cluster with B_c = 8 < U
    (dict(B=4, C=5), -2),                         # more clusters than rows
])
def test_create_rejects_invalid_descriptors_on_the_host(lib, kw, status):
    h = C.c_void_p(1)
    st = lib.cdm_create(C.byref(_desc(**kw)), C.byref(h))
    assert st == status
    assert h.value is None


@pytest.mark.parametrize("sizes,kw,status", [
    ([30, 30], dict(B=64, C=2), -2),                 # sizes do not sum to B
    ([64, 0], dict(B=64, C=2), -2),                  # an empty cluster
    ([40, -6, 30], dict(B=64, C=3), -2),             # a negative size
    ([50, 14], dict(B=64, U=16, C=2, problem=1), -6),  # downlink cluster with B_c = 14 < U
])
def test_create_rejects_invalid_cluster_sizes_on_the_host(lib, sizes, kw, status):
    arr = (C.c_int32 * len(sizes))(*sizes)
    d = _desc(**kw)
    d.Bc = C.cast(arr, C.POINTER(C.c_int32))
    h = C.c_void_p(1)
    assert lib.cdm_create(C.byref(d), C.byref(h)) == status
    assert h.value is None


def test_batched_plans_take_no_cluster_sizes(lib):
    m = np.array([64, 100], np.int32)
    n = np.array([32, 50], np.int32)
    arr = (C.c_int32 * 2)(32, 32)
    d = _desc(B=64, C=2)
    d.Bc = C.cast(arr, C.POINTER(C.c_int32))
    h = C.c_void_p(1)
    assert lib.cdm_create_batched(C.byref(d), 2, m.ctypes.data, n.ctypes.data, C.byref(h)) == -7
    assert h.value is None
    assert lib.cdm_create_batched(C.byref(_desc(C=2)), 2, m.ctypes.data, n.ctypes.data, C.byref(h)) == -7


def test_null_arguments(lib):
    assert lib.cdm_create(None, None) == -1
    assert lib.cdm_solve(None, None, 0, None, None, None, 0.1, 1.0, 0.0, None, None, None, None, None) == -1
    assert lib.cdm_destroy(None) == 0
    m = np.array([4], np.int32)
    assert lib.cdm_create_batched(C.byref(_desc()), 0, m.ctypes.data, m.ctypes.data,
                                  C.byref(C.c_void_p())) == -1
    # measurement utilities: NULL pointers and sizes that are not whole 16-byte words
    assert lib.cdm_stream_read(None, 16, None, None) == -1
    assert lib.cdm_stream_read(C.c_void_p(16), 24, C.c_void_p(16), None) == -1
    assert lib.cdm_stream_copy(C.c_void_p(16), C.c_void_p(32), -16, None) == -1


@pytest.mark.parametrize("kw,status", [
    (dict(precision=4, tol=0.0), -1),            # mixed refinement needs a tolerance
    (dict(precision=3, tol=1e-8), -7),           # FP8 inner copy: single solves only
    (dict(precision=2, tol=1e-8, problem=1), -7),
])
def test_create_batched_rejects_on_the_host(lib, kw, status):
    m = np.array([64, 100], np.int32)
    n = np.array([32, 50], np.int32)
    h = C.c_void_p(1)
    st = lib.cdm_create_batched(C.byref(_desc(**kw)), 2, m.ctypes.data, n.ctypes.data, C.byref(h))
    assert st == status
    assert h.value is None


def test_mixed_c64_is_batched_only(lib):
    h = C.c_void_p(1)
    assert lib.cdm_create(C.byref(_desc(precision=4, tol=1e-8)), C.byref(h)) == -7
    assert h.value is None


@pytest.mark.parametrize("args,status", [
    (dict(C=3), -2), (dict(Bc=33), -2), (dict(U=17), -2), (dict(U=0), -2), (dict(S=0), -2),
    (dict(prec=0), -3), (dict(T=0), -1), (dict(N0=-1.0), -1), (dict(Ex=0.0), -1),
    (dict(N0=0.0, Bc=4), -6),                     # lambda = 0 with B_c < U
])
def test_detect_batch_rejects_on_the_host(lib, args, status):
    a = dict(S=4, V=3, C=4, Bc=32, U=8, T=3, prec=1, N0=0.5, Ex=1.0)
    a.update(args)
    buf = C.c_void_p(16)   # never dereferenced: validation comes first
    st = lib.cdm_detect_batch(a["S"], a["V"], a["C"], a["Bc"], a["U"], a["T"], a["prec"], buf, buf,
                              a["N0"], a["Ex"], buf, None)
    assert st == status


@pytest.mark.parametrize("args,status", [
    (dict(C=3), -2), (dict(Bc=33), -2), (dict(U=17), -2), (dict(U=0), -2), (dict(S=0), -2),
    (dict(prec=0), -3), (dict(T=0), -1), (dict(rho=float("inf")), -1), (dict(Bc=4, U=8), -6),
])
def test_precode_batch_rejects_on_the_host(lib, args, status):
    a = dict(S=4, V=3, C=4, Bc=32, U=8, T=3, prec=1, rho=1.0)
    a.update(args)
    buf = C.c_void_p(16)   # never dereferenced: validation comes first
    st = lib.cdm_precode_batch(a["S"], a["V"], a["C"], a["Bc"], a["U"], a["T"], a["prec"], buf, buf,
                               a["rho"], buf, None)
    assert st == status


def test_info_record_layout():
    from paper_1902_08653_amd import cdm
    assert cdm.INFO_DTYPE.itemsize == 32
    assert C.sizeof(cdm.Desc) == 64
