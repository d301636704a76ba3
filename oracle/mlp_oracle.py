"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

Plain NumPy: three affine layers with ReLU after the first two, mean squared error
loss L = mean((Y - T)^2), and its gradients by the chain rule written out layer by
layer.  `bf16=True` rounds every product operand (layer inputs and weights) to BF16
(nearest even, from their FP32 value) the way the GPU's MFMA operands are formed,
so that the GPU result can be compared at the level of its FP32 accumulation.
Parameters use the same flat layout as the library: W1 (nin x h1), b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """FP64 -> FP32 (nearest) -> BF16 (nearest even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) >> 16
    out = (r.astype(np.uint32) << 16).view(np.float32)
    return out.astype(np.float64)


def split(flat, shape):
    nin, h1, h2, nout = shape
    sizes = [nin * h1, h1, h1 * h2, h2, h2 * nout, nout]
    shapes = [(nin, h1), (h1,), (h1, h2), (h2,), (h2, nout), (nout,)]
    out, k = [], 0
    for sz, sh in zip(sizes, shapes):
        out.append(np.asarray(flat[k:k + sz], dtype=np.float64).reshape(sh))
        k += sz
    return out


def _q(a, bf16):
    return bf16_round(a) if bf16 else np.asarray(a, dtype=np.float64)


def forward(flat, shape, X, bf16=False):
    W1, b1, W2, b2, W3, b3 = split(flat, shape)
    X = np.asarray(X, dtype=np.float64)
    Z1 = _q(X, bf16) @ _q(W1, bf16) + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = _q(A1, bf16) @ _q(W2, bf16) + b2
    A2 = np.maximum(Z2, 0.0)
    Y = _q(A2, bf16) @ _q(W3, bf16) + b3
    return dict(Z1=Z1, A1=A1, Z2=Z2, A2=A2, Y=Y)


def loss(flat, shape, X, T, bf16=False):
    Y = forward(flat, shape, X, bf16)["Y"]
    return float(np.mean((Y - np.asarray(T, dtype=np.float64)) ** 2))


def gradients(flat, shape, X, T, bf16=False):
    """dL/dparams (flat), L = mean over all rows and outputs of (Y - T)^2."""
    W1, b1, W2, b2, W3, b3 = split(flat, shape)
    f = forward(flat, shape, X, bf16)
    X = np.asarray(X, dtype=np.float64)
    Y = f["Y"]
    dY = 2.0 * (Y - np.asarray(T, dtype=np.float64)) / Y.size
    gW3 = _q(f["A2"], bf16).T @ _q(dY, bf16)
    gb3 = dY.sum(axis=0)
    dA2 = _q(dY, bf16) @ _q(W3, bf16).T
    dZ2 = dA2 * (f["Z2"] > 0)
    gW2 = _q(f["A1"], bf16).T @ _q(dZ2, bf16)
    gb2 = dZ2.sum(axis=0)
    dA1 = _q(dZ2, bf16) @ _q(W2, bf16).T
    dZ1 = dA1 * (f["Z1"] > 0)
    gW1 = _q(X, bf16).T @ _q(dZ1, bf16)
    gb1 = dZ1.sum(axis=0)
    return np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(w, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update (Kingma & Ba, Algorithm 1); returns (w, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m1, m2


def features(instances, lam):
    """Per-coordinate warm-start features of a list of (H (m x n complex), y (m)) pairs,
    rows in instance order then user order:
    [Re z, Im z, |z|, ||h_u||^2, lambda, m/2048, n/m, 1], z = h_u^H y / (||h_u||^2 + lambda)."""
    rows = []
    for H, y in instances:
        H = np.asarray(H, dtype=np.complex128)
        y = np.asarray(y, dtype=np.complex128)
        m, n = H.shape
        e = np.sum(np.abs(H) ** 2, axis=0)
        z = (H.conj().T @ y) / (e + lam)
        for u in range(n):
            rows.append([z[u].real, z[u].imag, abs(z[u]), e[u], lam, m / 2048.0, n / m, 1.0])
    return np.array(rows, dtype=np.float64).reshape(-1, 8)
