"""Thin Python binding of the C ABI in ``include/cdm.h`` (argument marshalling only).

Every step of the solve runs in the gfx950 kernels of ``libcdm.so``.  PyTorch is
used only to own device memory and to name the stream.  If the library is
missing this module raises on use; there is no fallback of any kind.

Channel layout: a B x U channel H is passed as a tensor ``Hc`` of shape (U, ld)
(contiguous): row u of ``Hc`` is user column h_u (column-major H, ld >= B).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# CDM_LIB names another build of the same library (the host-sanitizer build the CPU
# tests load); the default is the in-tree libcdm.so
LIB_PATH = os.environ.get("CDM_LIB") or os.path.join(_PKG, "libcdm.so")

UPLINK_LMMSE, DOWNLINK_ZF = 0, 1
C128, C64, MIXED_BF16, MIXED_FP8, MIXED_C64, C16 = 0, 1, 2, 3, 4, 5
DENSE, CSR = 0, 1
ENGINE_AUTO, ENGINE_WG, ENGINE_PANEL = 0, 1, 2
F_RESIDUAL = 1
F_TIMING = 2
F_AUTOTUNE = 4
F_NO_LOOKAHEAD = 8
F_DEEP_LOOKAHEAD = 16

INFO_ZERO_COLUMN, INFO_NONFINITE, INFO_NOT_CONVERGED, INFO_TIMEOUT = 1, 2, 4, 8

_PREC = {"c128": C128, "c64": C64, "bf16": MIXED_BF16, "fp8": MIXED_FP8, "mixed-c64": MIXED_C64}
_ENGINE = {"auto": ENGINE_AUTO, "wg": ENGINE_WG, "panel": ENGINE_PANEL}


class CdmError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = lib().cdm_status_string(status).decode()
        extra = lib().cdm_last_error().decode()
        super().__init__("%s: %s (%d)%s" % (where, msg, status, (" -- " + extra) if extra else ""))


class Desc(C.Structure):
    _fields_ = [("problem", C.c_int32), ("precision", C.c_int32), ("layout", C.c_int32),
                ("engine", C.c_int32), ("B", C.c_int32), ("U", C.c_int32), ("C", C.c_int32),
                ("T_max", C.c_int32), ("tol", C.c_double), ("nnz", C.c_int64),
                ("panel", C.c_int32), ("flags", C.c_int32), ("Bc", C.POINTER(C.c_int32))]


INFO_DTYPE = np.dtype([("sweeps", np.int32), ("flags", np.int32), ("rel_step", np.float64),
                       ("resid", np.float64), ("reserved", np.float64)])
assert INFO_DTYPE.itemsize == 32

EXPORTS = ["cdm_version", "cdm_status_string", "cdm_last_error", "cdm_create", "cdm_solve",
           "cdm_create_batched", "cdm_batched_offsets", "cdm_solve_batched", "cdm_residual",
           "cdm_plan_describe", "cdm_plan_timings", "cdm_stream_copy", "cdm_stream_read", "cdm_csr_transpose", "cdm_quantized_copy", "cdm_batched_features", "cdm_mlp_create",
           "cdm_mlp_param_count", "cdm_mlp_set_weights", "cdm_mlp_get_weights", "cdm_mlp_forward",
           "cdm_mlp_gradients", "cdm_mlp_train_step", "cdm_mlp_predict", "cdm_mlp_destroy", "cdm_destroy",
           "cdm_detect_batch", "cdm_precode_batch", "cdm_solve_noalloc"]

_lib = None


def lib():
    """Load libcdm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcdm.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.cdm_version.restype = i32
        L.cdm_status_string.argtypes = [i32]
        L.cdm_status_string.restype = C.c_char_p
        L.cdm_last_error.restype = C.c_char_p
        L.cdm_create.argtypes = [C.POINTER(Desc), C.POINTER(P)]
        L.cdm_create.restype = i32
        L.cdm_solve.argtypes = [P, P, i64, P, P, P, f64, f64, f64, P, P, P, P, P]
        L.cdm_solve.restype = i32
        L.cdm_solve_noalloc.argtypes = [C.POINTER(Desc), P, i64, P, f64, f64, f64, P, P, P, P, P]
        L.cdm_solve_noalloc.restype = i32
        L.cdm_create_batched.argtypes = [C.POINTER(Desc), i32, P, P, C.POINTER(P)]
        L.cdm_create_batched.restype = i32
        L.cdm_batched_offsets.argtypes = [P, P, P, P]
        L.cdm_batched_offsets.restype = i32
        L.cdm_solve_batched.argtypes = [P, P, P, f64, f64, P, P, P, P]
        L.cdm_solve_batched.restype = i32
        L.cdm_residual.argtypes = [P, P, i64, P, f64, f64, P, P, P]
        L.cdm_residual.restype = i32
        L.cdm_plan_describe.argtypes = [P, C.c_char_p, i32]
        L.cdm_plan_describe.restype = i32
        L.cdm_plan_timings.argtypes = [P, P, i32, P]
        L.cdm_plan_timings.restype = i32
        L.cdm_stream_copy.argtypes = [P, P, i64, P]
        L.cdm_stream_copy.restype = i32
        L.cdm_stream_read.argtypes = [P, i64, P, P]
        L.cdm_stream_read.restype = i32
        L.cdm_csr_transpose.argtypes = [P, P, P, P, P, P, P, P]
        L.cdm_csr_transpose.restype = i32
        L.cdm_quantized_copy.argtypes = [P, P, i64, P, P, P, P]
        L.cdm_quantized_copy.restype = i32
        L.cdm_batched_features.argtypes = [P, P, P, f64, f64, P, P]
        L.cdm_batched_features.restype = i32
        L.cdm_mlp_create.argtypes = [i32, i32, i32, i32, i32, C.POINTER(P)]
        L.cdm_mlp_create.restype = i32
        L.cdm_mlp_param_count.argtypes = [P]
        L.cdm_mlp_param_count.restype = i64
        L.cdm_mlp_set_weights.argtypes = [P, P, i64]
        L.cdm_mlp_set_weights.restype = i32
        L.cdm_mlp_get_weights.argtypes = [P, P, i64]
        L.cdm_mlp_get_weights.restype = i32
        L.cdm_mlp_forward.argtypes = [P, P, i32, P, P]
        L.cdm_mlp_forward.restype = i32
        L.cdm_mlp_gradients.argtypes = [P, P, P, i32, P, P, P]
        L.cdm_mlp_gradients.restype = i32
        L.cdm_mlp_train_step.argtypes = [P, P, P, i32, C.c_float, P]
        L.cdm_mlp_train_step.restype = i32
        L.cdm_mlp_predict.argtypes = [P, P, i64, P, i32, P]
        L.cdm_mlp_predict.restype = i32
        L.cdm_mlp_destroy.argtypes = [P]
        L.cdm_mlp_destroy.restype = i32
        L.cdm_destroy.argtypes = [P]
        L.cdm_destroy.restype = i32
        L.cdm_detect_batch.argtypes = [i32, i32, i32, i32, i32, i32, i32, P, P, f64, f64, P, P]
        L.cdm_detect_batch.restype = i32
        L.cdm_precode_batch.argtypes = [i32, i32, i32, i32, i32, i32, i32, P, P, f64, P, P]
        L.cdm_precode_batch.restype = i32
        _lib = L
    return _lib


def _check(st, where):
    if st != 0:
        raise CdmError(st, where)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def parse_info(info_tensor):
    """Device cdm_info records (uint8 tensor) -> structured NumPy array."""
    raw = info_tensor.detach().cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=INFO_DTYPE).copy()


def _cdtype(precision):
    import torch
    return torch.complex128 if precision in ("c128", "bf16", "fp8", "mixed-c64") else torch.complex64


class Plan:
    """A plan for single solves (``cdm_create`` / ``cdm_solve`` / ``cdm_destroy``).

    lookahead (dense panel engine): True, the look-ahead schedule (one panel ahead);
    "deep", two panels ahead where it applies (CDM_F_DEEP_LOOKAHEAD); False, the two-hop
    schedule (CDM_F_NO_LOOKAHEAD)."""

    def __init__(self, B, U, C_clusters=1, precision="c128", T_max=200, tol=0.0, engine="auto",
                 panel=0, residual=False, problem="uplink", layout="dense", nnz=0, timing=False,
                 lookahead=True, Bc=None):
        self.B, self.U, self.C = int(B), int(U), int(C_clusters)
        bc = None
        if Bc is not None:
            bc = (C.c_int32 * self.C)(*[int(v) for v in Bc])
        self.precision = precision
        self.problem = problem
        d = Desc(problem=UPLINK_LMMSE if problem == "uplink" else DOWNLINK_ZF,
                 precision=_PREC[precision], layout=DENSE if layout == "dense" else CSR,
                 engine=_ENGINE[engine], B=self.B, U=self.U, C=self.C, T_max=int(T_max),
                 tol=float(tol), nnz=int(nnz), panel=int(panel),
                 flags=(F_RESIDUAL if residual else 0) | (F_TIMING if timing else 0)
                 | (F_NO_LOOKAHEAD if lookahead is False else 0)
                 | (F_DEEP_LOOKAHEAD if lookahead == "deep" else 0),
                 Bc=C.cast(bc, C.POINTER(C.c_int32)) if bc is not None else None)
        self.desc = d
        h = C.c_void_p()
        _check(lib().cdm_create(C.byref(d), C.byref(h)), "cdm_create")
        self._h = h

    def describe(self):
        buf = C.create_string_buffer(1024)
        _check(lib().cdm_plan_describe(self._h, buf, 1024), "cdm_plan_describe")
        return buf.value.decode()

    def solve(self, Hc, rhs, N0=0.1, Ex=1.0, rho=0.0, x0=None, x=None, info=None, stream=None,
              rowptr=None, colidx=None, lambda_c=None):
        """Enqueue one solve.  Returns (x, info) device tensors; call parse_info(info)
        after synchronising to read the records.  lambda_c: optional device float64
        tensor of C fusion weights (used as given)."""
        import torch
        dev = rhs.device
        ldh = Hc.shape[1] if Hc.dim() == 2 else 0
        if x is None:
            n_out = self.U if self.problem == "uplink" else self.B
            x = torch.empty(n_out, dtype=rhs.dtype, device=dev)
        if info is None:
            info = torch.empty(32 * self.C, dtype=torch.uint8, device=dev)
        st = lib().cdm_solve(self._h, _ptr(Hc), int(ldh), _ptr(rowptr), _ptr(colidx), _ptr(rhs),
                             float(N0), float(Ex), float(rho), _ptr(x0), _ptr(lambda_c), _ptr(x),
                             _ptr(info), _stream(stream))
        _check(st, "cdm_solve")
        return x, info

    STAGES = ("preprocess", "init", "sweeps", "finalize")

    def timings(self):
        """Stage durations (ms) of the last solve (plan created with timing=True)."""
        out = np.zeros(4)
        cnt = C.c_int32(0)
        _check(lib().cdm_plan_timings(self._h, out.ctypes.data, 4, C.byref(cnt)), "cdm_plan_timings")
        return dict(zip(self.STAGES, out[:cnt.value].tolist()))

    def csr_transpose(self, val, rowptr, colidx, stream=None):
        """Column-compressed copy of a CSR channel (sparse plans): (colptr, rowidx, cval)."""
        import torch
        nnz = int(self.desc.nnz)
        colptr = torch.empty(self.U + 1, dtype=torch.int32, device=val.device)
        rowidx = torch.empty(max(nnz, 1), dtype=torch.int32, device=val.device)
        cval = torch.empty(max(nnz, 1), dtype=val.dtype, device=val.device)
        _check(lib().cdm_csr_transpose(self._h, _ptr(val), _ptr(rowptr), _ptr(colidx), _ptr(colptr),
                                       _ptr(rowidx), _ptr(cval), _stream(stream)), "cdm_csr_transpose")
        return colptr, rowidx[:nnz], cval[:nnz]

    def quantized_copy(self, Hc, stream=None):
        """Mixed plans: the planar low-precision copy of H (re, im[, block scales])."""
        import torch
        dt = torch.int16 if self.precision == "bf16" else torch.uint8
        re = torch.empty((self.U, self.B), dtype=dt, device=Hc.device)
        im = torch.empty_like(re)
        sc = torch.empty((self.U + 127) // 128, dtype=torch.float32, device=Hc.device)
        _check(lib().cdm_quantized_copy(self._h, _ptr(Hc), int(Hc.shape[1]), _ptr(re), _ptr(im), _ptr(sc),
                                        _stream(stream)), "cdm_quantized_copy")
        return (re, im) if self.precision == "bf16" else (re, im, sc)

    def residual(self, Hc, y, x, N0=0.1, Ex=1.0, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=y.device)
        _check(lib().cdm_residual(self._h, _ptr(Hc), int(Hc.shape[1]), _ptr(y), float(N0), float(Ex),
                                  _ptr(x), _ptr(out), _stream(stream)), "cdm_residual")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().cdm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_noalloc(Hc, rhs, B, U, C_clusters=1, Bc=None, precision="c128", T_max=3, tol=0.0,
                  problem="uplink", N0=0.1, Ex=1.0, rho=0.0, x0=None, lambda_c=None, x=None, info=None,
                  stream=None):
    """cdm_solve_noalloc: the per-cluster solve with the library's static scratch (no
    plan, no allocation inside the library).  x and info may be given to keep the call
    free of allocations on the Python side as well.  Returns (x, info)."""
    import torch
    Cn = int(C_clusters)
    bc = None if Bc is None else (C.c_int32 * Cn)(*[int(v) for v in Bc])
    d = Desc(problem=UPLINK_LMMSE if problem == "uplink" else DOWNLINK_ZF, precision=_PREC[precision],
             layout=DENSE, engine=ENGINE_AUTO, B=int(B), U=int(U), C=Cn, T_max=int(T_max), tol=float(tol),
             nnz=0, panel=0, flags=0, Bc=C.cast(bc, C.POINTER(C.c_int32)) if bc is not None else None)
    dev = rhs.device
    if x is None:
        x = torch.empty(int(U) if problem == "uplink" else int(B), dtype=rhs.dtype, device=dev)
    if info is None:
        info = torch.empty(32 * Cn, dtype=torch.uint8, device=dev)
    ldh = Hc.shape[1] if Hc.dim() == 2 else int(B)
    _check(lib().cdm_solve_noalloc(C.byref(d), _ptr(Hc), int(ldh), _ptr(rhs), float(N0), float(Ex), float(rho),
                                   _ptr(x0), _ptr(lambda_c), _ptr(x), _ptr(info), _stream(stream)),
           "cdm_solve_noalloc")
    return x, info


def detect_batch(H, Y, S, V, C_clusters, Bc, U, T_max, N0, Ex=1.0, out=None, stream=None):
    """cdm_detect_batch: fused decentralized detection of S subcarriers x V vectors.
    H, Y (and `out`) are device tensors of complex64, or of complex FP16 held as
    torch.complex32 / interleaved float16; returns X (S*V*U complex, Y's dtype)."""
    import torch
    if Y.dtype == torch.complex64:
        prec = C64
    elif Y.dtype in (torch.complex32, torch.float16):
        prec = C16
    else:
        raise TypeError("detect_batch takes complex64 or complex FP16 tensors")
    if H.dtype != Y.dtype:
        raise TypeError("H and Y must have the same dtype")
    per = 2 if Y.dtype == torch.float16 else 1
    if out is None:
        out = torch.empty(int(S) * int(V) * int(U) * per, dtype=Y.dtype, device=Y.device)
    _check(lib().cdm_detect_batch(int(S), int(V), int(C_clusters), int(Bc), int(U), int(T_max), prec, _ptr(H),
                                  _ptr(Y), float(N0), float(Ex), _ptr(out), _stream(stream)), "cdm_detect_batch")
    return out


def precode_batch(H, Sym, S, V, C_clusters, Bc, U, T_max, rho, out=None, stream=None):
    """cdm_precode_batch: decentralized ZF precoding of S subcarriers x V symbol
    vectors (Algorithm 2).  H, Sym (and `out`) are device tensors of complex64, or of
    complex FP16 held as torch.complex32 / interleaved float16; returns the stacked
    precoded vectors (S*V*B complex, B = C*Bc, Sym's dtype)."""
    import torch
    if Sym.dtype == torch.complex64:
        prec = C64
    elif Sym.dtype in (torch.complex32, torch.float16):
        prec = C16
    else:
        raise TypeError("precode_batch takes complex64 or complex FP16 tensors")
    if H.dtype != Sym.dtype:
        raise TypeError("H and Sym must have the same dtype")
    per = 2 if Sym.dtype == torch.float16 else 1
    if out is None:
        out = torch.empty(int(S) * int(V) * int(C_clusters) * int(Bc) * per, dtype=Sym.dtype, device=Sym.device)
    _check(lib().cdm_precode_batch(int(S), int(V), int(C_clusters), int(Bc), int(U), int(T_max), prec, _ptr(H),
                                   _ptr(Sym), float(rho), _ptr(out), _stream(stream)), "cdm_precode_batch")
    return out


def stream_copy(src, dst, stream=None):
    """Library copy kernel (measurement utility): dst[:] = src[:] (same byte size)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().cdm_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "cdm_stream_copy")


STREAM_READ_SLOTS = 8192
# inner sweeps per outer refinement step of a single mixed-precision solve
# (CDM_MIXED_INNER_SWEEPS_BF16 / _FP8)
MIXED_INNER_SWEEPS = {"bf16": 12, "fp8": 5}


def stream_read(src, out, stream=None):
    """Library read-only stream (measurement utility): out (STREAM_READ_SLOTS x 16 bytes
    on the device) receives partial XORs whose XOR is that of every 16-byte word of src."""
    nbytes = src.numel() * src.element_size()
    assert out.numel() * out.element_size() == 16 * STREAM_READ_SLOTS
    _check(lib().cdm_stream_read(_ptr(src), int(nbytes), _ptr(out), _stream(stream)), "cdm_stream_read")


class BatchedPlan:
    """A plan for many independent uplink instances of uneven size."""

    def __init__(self, m, n, precision="c64", T_max=200, tol=0.0, residual=False, autotune=False):
        m = np.ascontiguousarray(m, dtype=np.int32)
        n = np.ascontiguousarray(n, dtype=np.int32)
        self.batch = int(m.shape[0])
        self.m, self.n = m, n
        self.precision = precision
        d = Desc(problem=UPLINK_LMMSE, precision=_PREC[precision], layout=DENSE, engine=ENGINE_WG,
                 B=int(m.max()), U=int(n.max()), C=1, T_max=int(T_max), tol=float(tol), nnz=0,
                 panel=0, flags=(F_RESIDUAL if residual else 0) | (F_AUTOTUNE if autotune else 0))
        h = C.c_void_p()
        _check(lib().cdm_create_batched(C.byref(d), self.batch, m.ctypes.data, n.ctypes.data,
                                        C.byref(h)), "cdm_create_batched")
        self._h = h
        self.H_off = np.zeros(self.batch, np.int64)
        self.y_off = np.zeros(self.batch, np.int64)
        self.x_off = np.zeros(self.batch, np.int64)
        _check(lib().cdm_batched_offsets(h, self.H_off.ctypes.data, self.y_off.ctypes.data,
                                         self.x_off.ctypes.data), "cdm_batched_offsets")

    def describe(self):
        buf = C.create_string_buffer(1024)
        _check(lib().cdm_plan_describe(self._h, buf, 1024), "cdm_plan_describe")
        return buf.value.decode()

    def features(self, H, y, N0=0.1, Ex=1.0, out=None, stream=None):
        """Per-coordinate feature rows (sum n_i x 8 float32) of the packed batch."""
        import torch
        F = out
        if F is None:
            F = torch.empty((int(self.n.astype(np.int64).sum()), 8), dtype=torch.float32, device=y.device)
        _check(lib().cdm_batched_features(self._h, _ptr(H), _ptr(y), float(N0), float(Ex), _ptr(F),
                                          _stream(stream)), "cdm_batched_features")
        return F

    def solve(self, H, y, N0=0.1, Ex=1.0, x0=None, x=None, info=None, stream=None):
        import torch
        if x is None:
            x = torch.empty(int(self.n.astype(np.int64).sum()), dtype=y.dtype, device=y.device)
        if info is None:
            info = torch.empty(32 * self.batch, dtype=torch.uint8, device=y.device)
        _check(lib().cdm_solve_batched(self._h, _ptr(H), _ptr(y), float(N0), float(Ex), _ptr(x0),
                                       _ptr(x), _ptr(info), _stream(stream)), "cdm_solve_batched")
        return x, info

    def close(self):
        if getattr(self, "_h", None):
            lib().cdm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Mlp:
    """The warm-start network (cdm_mlp_*): nin -> h1 -> h2 -> nout, ReLU, BF16 MFMA."""

    def __init__(self, nin=8, h1=512, h2=512, nout=2, max_rows=8192):
        h = C.c_void_p()
        _check(lib().cdm_mlp_create(int(nin), int(h1), int(h2), int(nout), int(max_rows), C.byref(h)),
               "cdm_mlp_create")
        self._h = h
        self.shape = (nin, h1, h2, nout)
        self.max_rows = max_rows
        self.nparam = int(lib().cdm_mlp_param_count(h))

    def split(self, flat):
        nin, h1, h2, nout = self.shape
        sizes = [nin * h1, h1, h1 * h2, h2, h2 * nout, nout]
        shapes = [(nin, h1), (h1,), (h1, h2), (h2,), (h2, nout), (nout,)]
        out, k = [], 0
        for sz, sh in zip(sizes, shapes):
            out.append(np.asarray(flat[k:k + sz]).reshape(sh))
            k += sz
        return out

    def init(self, seed=0):
        """He-style initialisation from a seeded generator (host), uploaded."""
        rng = np.random.default_rng(seed)
        nin, h1, h2, nout = self.shape
        parts = [rng.standard_normal((nin, h1)) * np.sqrt(2.0 / nin), np.zeros(h1),
                 rng.standard_normal((h1, h2)) * np.sqrt(2.0 / h1), np.zeros(h2),
                 rng.standard_normal((h2, nout)) * np.sqrt(1.0 / h2), np.zeros(nout)]
        self.set_weights(np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32))

    def set_weights(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().cdm_mlp_set_weights(self._h, flat.ctypes.data, self.nparam), "cdm_mlp_set_weights")

    def get_weights(self):
        out = np.zeros(self.nparam, np.float32)
        _check(lib().cdm_mlp_get_weights(self._h, out.ctypes.data, self.nparam), "cdm_mlp_get_weights")
        return out

    def forward(self, X, Y=None, stream=None):
        import torch
        if Y is None:
            Y = torch.empty((X.shape[0], self.shape[3]), dtype=torch.float32, device=X.device)
        _check(lib().cdm_mlp_forward(self._h, _ptr(X), int(X.shape[0]), _ptr(Y), _stream(stream)),
               "cdm_mlp_forward")
        return Y

    def gradients(self, X, T, stream=None):
        import torch
        g = torch.empty(self.nparam, dtype=torch.float32, device=X.device)
        parts = torch.empty((X.shape[0] * self.shape[3] + 255) // 256, dtype=torch.float32, device=X.device)
        _check(lib().cdm_mlp_gradients(self._h, _ptr(X), _ptr(T), int(X.shape[0]), _ptr(g), _ptr(parts),
                                       _stream(stream)), "cdm_mlp_gradients")
        return g, parts

    def train_step(self, X, T, lr, stream=None):
        _check(lib().cdm_mlp_train_step(self._h, _ptr(X), _ptr(T), int(X.shape[0]), float(lr),
                                        _stream(stream)), "cdm_mlp_train_step")

    def predict(self, X, dtype, out=None, stream=None):
        """Warm start x0 (complex `dtype`, one entry per feature row) from the network."""
        import torch
        if out is None:
            out = torch.empty(X.shape[0], dtype=dtype, device=X.device)
        prec = _PREC["c128" if dtype == torch.complex128 else "c64"]
        _check(lib().cdm_mlp_predict(self._h, _ptr(X), int(X.shape[0]), _ptr(out), prec, _stream(stream)),
               "cdm_mlp_predict")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().cdm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
