"""Learned warm start for the batched uplink solve.

A per-coordinate network maps cheap problem-data features of user u (its
regularised matched-filter estimate, column energy, lambda and the instance shape;
cdm_batched_features) to a starting point x_u^(0) for Algorithm 1.  CD converges
from any start (Sec. III-B: it is Gauss-Seidel on a positive definite system), so a
start closer to the solution only shortens the sweep count; the result is the same
stationary point.

Everything on the device path runs in the library's kernels: the feature pass, the
network (BF16 MFMA GEMMs), its training step and the conversion of its output into
the complex x0 that cdm_solve_batched takes.  This module only schedules the calls
and keeps the training data.
"""
from __future__ import annotations

import time

import numpy as np

from . import cdm

NFEAT = 8


class WarmStart:
    """The network plus its training loop (Adam on mean squared error)."""

    def __init__(self, hidden=512, max_rows=16384, seed=0):
        self.net = cdm.Mlp(NFEAT, hidden, hidden, 2, max_rows)
        self.net.init(seed)
        self.max_rows = max_rows

    # -- data -------------------------------------------------------------------
    @staticmethod
    def training_rows(plan, H, y, x_star, N0=0.1, Ex=1.0):
        """(features, targets) of one solved batch: targets are (Re, Im) of the
        solution as FP32 rows, in the packed x order."""
        import torch
        F = plan.features(H, y, N0, Ex)
        T = torch.view_as_real(x_star).to(torch.float32).contiguous()
        return F, T

    # -- training ---------------------------------------------------------------
    def fit(self, F, T, epochs=3, batch=None, lr=1e-3, seed=0, log=None):
        """Adam over shuffled mini-batches; returns the mean training loss per epoch."""
        import torch
        batch = batch or self.max_rows
        n = F.shape[0]
        g = torch.Generator(device="cpu")
        g.manual_seed(seed)
        perm = torch.randperm(n, generator=g).to(F.device)
        F = F[perm].contiguous()
        T = T[perm].contiguous()
        starts = np.arange(0, n, batch)
        rng = np.random.default_rng(seed)
        hist = []
        for ep in range(epochs):
            t0 = time.perf_counter()
            rng.shuffle(starts)
            tot = torch.zeros((), dtype=torch.float64, device=F.device)
            cnt = 0
            for k, s in enumerate(starts):
                e = min(n, int(s) + batch)
                self.net.train_step(F[s:e], T[s:e], lr)
                if k % 16 == 0:    # sample the loss of every 16th mini-batch
                    _, parts = self.net.gradients(F[s:e], T[s:e])
                    tot += parts.double().sum() / ((e - s) * 2)
                    cnt += 1
            hist.append(float(tot) / max(cnt, 1))
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.5f} ({time.perf_counter() - t0:.1f} s)")
        return hist

    def loss(self, F, T):
        """Mean squared error of the network on (F, T), evaluated in chunks."""
        tot = 0.0
        for s in range(0, F.shape[0], self.max_rows):
            e = min(F.shape[0], s + self.max_rows)
            _, parts = self.net.gradients(F[s:e], T[s:e])
            tot += float(parts.double().sum())
        return tot / (F.shape[0] * 2)

    # -- use --------------------------------------------------------------------
    def x0(self, plan, H, y, N0=0.1, Ex=1.0, out=None, feat=None, stream=None):
        """Feature pass + network: the warm start of every packed coordinate.  With
        preallocated `out` and `feat` buffers nothing is allocated (graph capture)."""
        F = plan.features(H, y, N0, Ex, out=feat, stream=stream)
        return self.net.predict(F, y.dtype, out=out, stream=stream)

    def solve(self, plan, H, y, N0=0.1, Ex=1.0, x0=None, feat=None, x=None, info=None, stream=None):
        x0 = self.x0(plan, H, y, N0, Ex, out=x0, feat=feat, stream=stream)
        return plan.solve(H, y, N0, Ex, x0=x0, x=x, info=info, stream=stream)

    def close(self):
        self.net.close()
