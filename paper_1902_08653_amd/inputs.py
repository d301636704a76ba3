"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic.  Both the GPU path and the CPU oracle consume exactly these
arrays.  All draws use NumPy's PCG64 ``default_rng(seed)``.

Channel model (Sec. II-A): H is B x U complex with i.i.d. circularly symmetric
Gaussian entries.  The dense instances here use variance 1/B per entry (real and
imaginary parts N(0, 1/(2B))), so E||h_u||^2 = 1; vectors are CN(0, 1).

Layout: a B x U channel is drawn as a (U, B) C-order array (column u of H is row
u of the draw), so the draw itself is column-major H with leading dimension B.
Draw order: Re(H), Im(H), Re(y), Im(y).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class DenseInstance:
    H: np.ndarray      # (B, U) view, Fortran-contiguous (column-major); H.T is C-contiguous
    y: np.ndarray      # (B,)
    seed: int

    @property
    def B(self):
        return self.H.shape[0]

    @property
    def U(self):
        return self.H.shape[1]


def dense_uplink(B: int, U: int, seed: int, var_h: float | None = None,
                 dtype=np.complex128) -> DenseInstance:
    """H ~ CN(0, var_h) (default 1/B), y ~ CN(0, 1).  Draw order Re(H), Im(H), Re(y), Im(y)."""
    rng = np.random.default_rng(seed)
    vh = (1.0 / B) if var_h is None else var_h
    sd = np.sqrt(vh / 2.0)
    Ht = np.empty((U, B), dtype=np.complex128)
    Ht.real = rng.standard_normal((U, B)) * sd
    Ht.imag = rng.standard_normal((U, B)) * sd
    y = np.empty(B, dtype=np.complex128)
    y.real = rng.standard_normal(B) * np.sqrt(0.5)
    y.imag = rng.standard_normal(B) * np.sqrt(0.5)
    if dtype != np.complex128:
        Ht = Ht.astype(np.complex64)
        y = y.astype(np.complex64)
    return DenseInstance(H=Ht.T, y=y, seed=seed)


@dataclass
class CsrInstance:
    B: int
    U: int
    rowptr: np.ndarray   # int32 (B+1)
    colidx: np.ndarray   # int32 (nnz), strictly increasing within each row
    val: np.ndarray      # complex (nnz)
    y: np.ndarray
    seed: int

    def dense(self):
        H = np.zeros((self.B, self.U), dtype=self.val.dtype, order="F")
        for i in range(self.B):
            a, b = self.rowptr[i], self.rowptr[i + 1]
            H[i, self.colidx[a:b]] = self.val[a:b]
        return H


def sparse_uplink(B: int, U: int, density: float, seed: int, scale_to_unit_column: bool = True,
                  dtype=np.complex128) -> CsrInstance:
    """Bernoulli(density) pattern, uniform random; nonzeros CN(0, v) with
    v = 1/(density*B) (so E||h_u||^2 = 1) or v = 1/B when ``scale_to_unit_column``
    is false.  Draw order: pattern (one uniform per entry, row by row in blocks),
    Re(val), Im(val), Re(y), Im(y)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    blk = max(1, (1 << 24) // max(U, 1))
    for r0 in range(0, B, blk):
        r1 = min(B, r0 + blk)
        mask = rng.random((r1 - r0, U)) < density
        rr, cc = np.nonzero(mask)          # row-major order: rows ascending, cols ascending
        rows.append(rr.astype(np.int64) + r0)
        cols.append(cc.astype(np.int64))
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    nnz = rows.shape[0]
    v = (1.0 / (density * B)) if scale_to_unit_column else (1.0 / B)
    sd = np.sqrt(v / 2.0)
    val = np.empty(nnz, np.complex128)
    val.real = rng.standard_normal(nnz) * sd
    val.imag = rng.standard_normal(nnz) * sd
    y = np.empty(B, np.complex128)
    y.real = rng.standard_normal(B) * np.sqrt(0.5)
    y.imag = rng.standard_normal(B) * np.sqrt(0.5)
    rowptr = np.zeros(B + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    if dtype != np.complex128:
        val = val.astype(np.complex64)
        y = y.astype(np.complex64)
    return CsrInstance(B=B, U=U, rowptr=rowptr, colidx=cols.astype(np.int32), val=val, y=y,
                       seed=seed)


def batch_sizes(count: int, seed0: int = 0, m_lo: int = 64, m_hi: int = 2048):
    """Instance i draws m_i ~ U{m_lo..m_hi} first from its own default_rng(seed0 + i);
    n_i = m_i // 2."""
    ms = np.empty(count, np.int32)
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        ms[i] = rng.integers(m_lo, m_hi + 1)
    return ms, (ms // 2).astype(np.int32)


def batch_instance(i: int, seed0: int = 0, m_lo: int = 64, m_hi: int = 2048,
                   dtype=np.complex128):
    """Instance i of the uneven batch: after drawing m (above), H ~ CN(0, 1/m), y ~ CN(0, 1)
    from the same generator; draw order m, Re(H) (n, m), Im(H), Re(y), Im(y)."""
    rng = np.random.default_rng(seed0 + i)
    m = int(rng.integers(m_lo, m_hi + 1))
    n = m // 2
    sd = np.sqrt(0.5 / m)
    Ht = np.empty((n, m), np.complex128)
    Ht.real = rng.standard_normal((n, m)) * sd
    Ht.imag = rng.standard_normal((n, m)) * sd
    y = np.empty(m, np.complex128)
    y.real = rng.standard_normal(m) * np.sqrt(0.5)
    y.imag = rng.standard_normal(m) * np.sqrt(0.5)
    if dtype != np.complex128:
        Ht = Ht.astype(np.complex64)
        y = y.astype(np.complex64)
    return DenseInstance(H=Ht.T, y=y, seed=seed0 + i)


def pack_batch(instances, dtype=np.complex128):
    """Pack instances back to back: H_i column-major with ld = m_i, in instance order;
    y_i and x_i likewise.  Returns (H_flat, y_flat, m, n, H_off, y_off, x_off)."""
    m = np.array([ins.B for ins in instances], np.int32)
    n = np.array([ins.U for ins in instances], np.int32)
    hsz = m.astype(np.int64) * n.astype(np.int64)
    H_off = np.concatenate([[0], np.cumsum(hsz)[:-1]]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum(m.astype(np.int64))[:-1]]).astype(np.int64)
    x_off = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]]).astype(np.int64)
    Hf = np.empty(int(hsz.sum()), dtype)
    yf = np.empty(int(m.astype(np.int64).sum()), dtype)
    for k, ins in enumerate(instances):
        Hf[H_off[k]:H_off[k] + hsz[k]] = ins.H.T.reshape(-1)
        yf[y_off[k]:y_off[k] + m[k]] = ins.y
    return Hf, yf, m, n, H_off, y_off, x_off


def batch_uneven_device(count: int, seed0: int = 0, m_lo: int = 64, m_hi: int = 2048, dtype=None,
                        device="cuda:0"):
    """The uneven batch drawn directly in device memory (for sizes too large to draw
    on the host): instance sizes m_i, n_i = m_i // 2 exactly as batch_sizes(); the
    packed H (instance by instance, column-major, ld = m_i) and y come from torch's
    device generator seeded with seed0: H_i ~ CN(0, 1/m_i), y ~ CN(0, 1).
    Returns (H, y, m, n) with H and y device tensors."""
    import torch
    dtype = torch.complex64 if dtype is None else dtype
    m, n = batch_sizes(count, seed0, m_lo, m_hi)
    hsz = m.astype(np.int64) * n.astype(np.int64)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed0) + 7919)
    H = torch.randn(int(hsz.sum()), dtype=dtype, device=device, generator=g)
    y = torch.randn(int(m.astype(np.int64).sum()), dtype=dtype, device=device, generator=g)
    off = 0
    for i in range(count):
        H[off:off + int(hsz[i])].mul_(float(1.0 / np.sqrt(m[i])))
        off += int(hsz[i])
    return H, y, m, n


# 16-QAM with unit average energy (Gray mapping on each axis): the paper's
# simulations and throughput figures use 16-QAM (Sec. V, Sec. VI-C).
QAM16_LEVELS = np.array([-3.0, -1.0, 3.0, 1.0]) / np.sqrt(10.0)   # index = 2 Gray bits


def qam16_symbols(bits: np.ndarray) -> np.ndarray:
    """Map a (..., 4) array of bits to 16-QAM symbols (bits 0-1 -> I, bits 2-3 -> Q)."""
    bi = bits[..., 0] * 2 + bits[..., 1]
    bq = bits[..., 2] * 2 + bits[..., 3]
    return QAM16_LEVELS[bi] + 1j * QAM16_LEVELS[bq]


def paper_shaped(C: int, Bc: int, U: int, n_sc: int, n_sym: int, snr_db: float, seed: int,
                 dtype=np.complex64):
    """Decentralised uplink workload of the paper's throughput experiment
    (Sec. VI-C): per subcarrier a Rayleigh channel H (B x U, B = C*Bc, entries
    CN(0, 1)), n_sym 16-QAM vectors x (Ex = 1) and y = H x + n with N0 = U/SNR
    (per-antenna SNR over the U streams).  Returns H as (n_sc, U, B) C-order
    (column-major per subcarrier), X (n_sc, n_sym, U), Y (n_sc, n_sym, B), bits, N0.
    """
    rng = np.random.default_rng(seed)
    B = C * Bc
    Ht = (rng.standard_normal((n_sc, U, B)) + 1j * rng.standard_normal((n_sc, U, B))) * np.sqrt(0.5)
    bits = rng.integers(0, 2, size=(n_sc, n_sym, U, 4), dtype=np.int8)
    X = qam16_symbols(bits)
    N0 = U / (10.0 ** (snr_db / 10.0))
    noise = (rng.standard_normal((n_sc, n_sym, B)) + 1j * rng.standard_normal((n_sc, n_sym, B))) \
        * np.sqrt(N0 / 2.0)
    Y = np.einsum("sub,snu->snb", Ht, X) + noise
    return dict(Ht=Ht.astype(dtype), X=X, Y=Y.astype(dtype), bits=bits, N0=N0, B=B)
