"""Python face of the FP64 CPU oracle (``cd_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  The product library never loads it; it shares no code with
the GPU path.

Every function takes NumPy arrays in the uplink orientation of Sec. II-A of the
paper: ``H`` is B x U (any NumPy layout; it is passed column-major), ``y`` is a
length-B complex vector, ``lambda = N0 / Ex`` is the regulariser of eq. (1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cd_oracle.c")
# CDO_SANITIZE=1: an AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# source (loaded into a process started with libasan preloaded; see
# tests/test_sanitizers.py), kept apart from the plain build
_SANITIZE = os.environ.get("CDO_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
# clang instruments every load, including those of `double complex` elements, which
# gcc's AddressSanitizer leaves unchecked; the shared sanitizer runtime is preloaded
SAN_CC = "/opt/rocm/llvm/bin/clang"
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-shared-libsan",
              "-fno-sanitize-recover=all"]


def sanitizer_runtime():
    """Path of the shared ASan (+UBSan) runtime that a process loading the sanitized
    oracle must preload, or None where the compiler is absent."""
    if not os.path.exists(SAN_CC):
        return None
    path = subprocess.check_output([SAN_CC, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None

FLAG_ZERO_COLUMN = 1
FLAG_NONFINITE = 2
FLAG_NOT_CONVERGED = 4


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no BLAS).

    ``-fcx-limited-range`` makes complex products the textbook four-multiply
    formula instead of a library call with Annex-G Inf recovery; the values are
    identical for finite inputs.
    """
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cc, opt = (SAN_CC, _SAN_FLAGS) if _SANITIZE else ("gcc", ["-O2"])
        subprocess.check_call([cc] + opt + ["-std=c99", "-fcx-limited-range", "-fPIC", "-shared",
                                            _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        i32, i64, f64 = C.c_int, C.c_long, C.c_double
        _lib.cdo_column_scalars.argtypes = [i32, i32, P, i64, f64, P, P, P]
        _lib.cdo_column_scalars.restype = None
        _lib.cdo_local_cd.argtypes = [i32, i32, P, i64, P, f64, P, i32, f64, P, P, P, P, P, P, P]
        _lib.cdo_local_cd.restype = i32
        _lib.cdo_uplink_cd.argtypes = [i32, i32, i32, P, P, i64, P, f64, f64, P, P, i32, f64,
                                       P, P, P, P, P, P]
        _lib.cdo_uplink_cd.restype = i32
        _lib.cdo_local_zf_cd.argtypes = [i32, i32, P, i64, P, i32, f64, P, P, P, P, P]
        _lib.cdo_local_zf_cd.restype = i32
        _lib.cdo_downlink_cd.argtypes = [i32, i32, i32, P, P, i64, P, f64, i32, f64, P, P, P, P]
        _lib.cdo_downlink_cd.restype = i32
        _lib.cdo_csr_to_csc.argtypes = [i32, i32, P, P, P, P, P, P]
        _lib.cdo_csr_to_csc.restype = None
        _lib.cdo_local_cd_csc.argtypes = [i32, i32, P, P, P, P, f64, P, i32, f64, P, P, P]
        _lib.cdo_local_cd_csc.restype = i32
        _lib.cdo_normal_residual.argtypes = [i32, i32, P, i64, P, f64, P]
        _lib.cdo_normal_residual.restype = f64
        _lib.cdo_bf16_code.argtypes = [f64]
        _lib.cdo_bf16_code.restype = C.c_uint16
        _lib.cdo_e4m3_code.argtypes = [C.c_float]
        _lib.cdo_e4m3_code.restype = C.c_uint8
        _lib.cdo_e4m3_value.argtypes = [C.c_uint8]
        _lib.cdo_e4m3_value.restype = f64
        _lib.cdo_quantize.argtypes = [i32, i32, i32, P, i64, P, P, P, P, P]
        _lib.cdo_quantize.restype = None
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _colmajor(H):
    H = np.asarray(H, dtype=np.complex128)
    return np.asfortranarray(H)


def _vec(v, n=None):
    v = np.ascontiguousarray(np.asarray(v, dtype=np.complex128).reshape(-1))
    if n is not None and v.shape[0] != n:
        raise ValueError("vector length %d, expected %d" % (v.shape[0], n))
    return v


def column_scalars(H, lam):
    """Alg. 1 preprocessing: (e_u, m_u, n_u) for every column of H."""
    H = _colmajor(H)
    B, U = H.shape
    e, m, n = (np.zeros(U) for _ in range(3))
    lib().cdo_column_scalars(B, U, _ptr(H), max(B, 1), float(lam), _ptr(e), _ptr(m), _ptr(n))
    return e, m, n


def local_cd(H, y, lam, T_max, tol=0.0, x0=None, trace=False):
    """Alg. 1 local CD at one cluster.

    Returns a dict with ``x``, ``sweeps``, ``rel_step``, ``flags`` and, when
    ``trace`` is true, ``sweep_x`` (T x U), ``step_x`` (T x U x U), ``step_r``
    (T x U x B) and ``sweep_s`` (T).
    """
    H = _colmajor(H)
    B, U = H.shape
    y = _vec(y, B)
    x0 = None if x0 is None else _vec(x0, U)
    x = np.zeros(U, np.complex128)
    rel = C.c_double(0.0)
    fl = C.c_int(0)
    tr = {}
    if trace:
        tr = dict(sweep_x=np.zeros((T_max, U), np.complex128),
                  step_x=np.zeros((T_max, U, U), np.complex128),
                  step_r=np.zeros((T_max, U, B), np.complex128),
                  sweep_s=np.zeros(T_max))
    t = lib().cdo_local_cd(B, U, _ptr(H), max(B, 1), _ptr(y), float(lam), _ptr(x0), int(T_max),
                           float(tol), _ptr(x), C.byref(rel), C.byref(fl),
                           _ptr(tr.get("sweep_x")), _ptr(tr.get("step_x")),
                           _ptr(tr.get("step_r")), _ptr(tr.get("sweep_s")))
    out = dict(x=x, sweeps=int(t), rel_step=rel.value, flags=fl.value)
    if trace:
        for k, v in tr.items():
            out[k] = v[:t]
    return out


def uplink_cd(H, y, N0, Ex, T_max, tol=0.0, C_clusters=1, Bc=None, x0=None, lam_c=None):
    """Alg. 1 end to end (clusters, local CD, fusion)."""
    H = _colmajor(H)
    B, U = H.shape
    y = _vec(y, B)
    Cn = int(C_clusters)
    bc = None
    if Bc is not None:
        bc = np.ascontiguousarray(np.asarray(Bc, dtype=np.int32))
        if bc.shape[0] != Cn or int(bc.sum()) != B:
            raise ValueError("cluster sizes must sum to B")
    elif B % Cn:
        raise ValueError("B must be divisible by C when Bc is not given")
    x0 = None if x0 is None else _vec(x0, U)
    lc = None if lam_c is None else np.ascontiguousarray(np.asarray(lam_c, dtype=np.float64))
    xh = np.zeros(U, np.complex128)
    xl = np.zeros((Cn, U), np.complex128)
    sw = np.zeros(Cn, np.int32)
    rs = np.zeros(Cn)
    fl = np.zeros(Cn, np.int32)
    wts = np.zeros(Cn)
    lib().cdo_uplink_cd(B, U, Cn, _ptr(bc), _ptr(H), max(B, 1), _ptr(y), float(N0), float(Ex),
                        _ptr(x0), _ptr(lc), int(T_max), float(tol), _ptr(xh), _ptr(xl),
                        _ptr(sw), _ptr(rs), _ptr(fl), _ptr(wts))
    return dict(x=xh, x_local=xl, sweeps=sw, rel_step=rs, flags=fl, weights=wts)


def local_zf_cd(H, s, T_max, tol=0.0, trace=False):
    """Alg. 2 / eq. (4) local CD at one cluster (no power scaling)."""
    H = _colmajor(H)
    B, U = H.shape
    s = _vec(s, U)
    x = np.zeros(B, np.complex128)
    rel = C.c_double(0.0)
    fl = C.c_int(0)
    tr = {}
    if trace:
        tr = dict(sweep_x=np.zeros((T_max, B), np.complex128),
                  step_x=np.zeros((T_max, U, B), np.complex128))
    t = lib().cdo_local_zf_cd(B, U, _ptr(H), max(B, 1), _ptr(s), int(T_max), float(tol), _ptr(x),
                              C.byref(rel), C.byref(fl), _ptr(tr.get("sweep_x")),
                              _ptr(tr.get("step_x")))
    out = dict(x=x, sweeps=int(t), rel_step=rel.value, flags=fl.value)
    if trace:
        for k, v in tr.items():
            out[k] = v[:t]
    return out


def downlink_cd(H, s, rho, T_max, tol=0.0, C_clusters=1, Bc=None):
    """Alg. 2 end to end (broadcast s, local CD, local power scaling, stacking)."""
    H = _colmajor(H)
    B, U = H.shape
    s = _vec(s, U)
    Cn = int(C_clusters)
    bc = None
    if Bc is not None:
        bc = np.ascontiguousarray(np.asarray(Bc, dtype=np.int32))
    elif B % Cn:
        raise ValueError("B must be divisible by C when Bc is not given")
    x = np.zeros(B, np.complex128)
    sw = np.zeros(Cn, np.int32)
    rs = np.zeros(Cn)
    fl = np.zeros(Cn, np.int32)
    lib().cdo_downlink_cd(B, U, Cn, _ptr(bc), _ptr(H), max(B, 1), _ptr(s), float(rho), int(T_max),
                          float(tol), _ptr(x), _ptr(sw), _ptr(rs), _ptr(fl))
    return dict(x=x, sweeps=sw, rel_step=rs, flags=fl)


def csr_to_csc(B, U, rowptr, colidx, val):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    val = _vec(val)
    nnz = int(rowptr[-1])
    colptr = np.zeros(U + 1, np.int32)
    rowidx = np.zeros(max(nnz, 1), np.int32)
    cval = np.zeros(max(nnz, 1), np.complex128)
    lib().cdo_csr_to_csc(B, U, _ptr(rowptr), _ptr(colidx), _ptr(val), _ptr(colptr), _ptr(rowidx),
                         _ptr(cval))
    return colptr, rowidx[:nnz], cval[:nnz]


def local_cd_csc(B, U, colptr, rowidx, cval, y, lam, T_max, tol=0.0, x0=None):
    colptr = np.ascontiguousarray(colptr, dtype=np.int32)
    rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
    cval = _vec(cval)
    y = _vec(y, B)
    x0 = None if x0 is None else _vec(x0, U)
    x = np.zeros(U, np.complex128)
    rel = C.c_double(0.0)
    fl = C.c_int(0)
    t = lib().cdo_local_cd_csc(B, U, _ptr(colptr), _ptr(rowidx), _ptr(cval), _ptr(y), float(lam),
                               _ptr(x0), int(T_max), float(tol), _ptr(x), C.byref(rel),
                               C.byref(fl))
    return dict(x=x, sweeps=int(t), rel_step=rel.value, flags=fl.value)


def normal_residual(H, y, lam, x):
    H = _colmajor(H)
    B, U = H.shape
    y = _vec(y, B)
    x = _vec(x, U)
    return lib().cdo_normal_residual(B, U, _ptr(H), max(B, 1), _ptr(y), float(lam), _ptr(x))


def quantize(H, kind):
    """Planar low-precision copy of H (see cd_oracle.c): kind "bf16" -> (re, im) uint16
    arrays of shape (U, B); kind "fp8" -> (re, im) uint8 arrays and the block scales."""
    H = _colmajor(H)
    B, U = H.shape
    if kind == "bf16":
        re = np.zeros((U, B), np.uint16)
        im = np.zeros((U, B), np.uint16)
        lib().cdo_quantize(0, B, U, _ptr(H), max(B, 1), _ptr(re), _ptr(im), None, None, None)
        return re, im
    re = np.zeros((U, B), np.uint8)
    im = np.zeros((U, B), np.uint8)
    sc = np.zeros((U + 127) // 128, np.float32)
    lib().cdo_quantize(1, B, U, _ptr(H), max(B, 1), None, None, _ptr(re), _ptr(im), _ptr(sc))
    return re, im, sc


def e4m3_value(code):
    return lib().cdo_e4m3_value(int(code))


def e4m3_code(v):
    return int(lib().cdo_e4m3_code(float(v)))


def bf16_code(v):
    return int(lib().cdo_bf16_code(float(v)))
