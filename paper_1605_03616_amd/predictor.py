"""Learned Chebyshev-order predictor: training data, training, order choice.

The training data come from the factorization itself: for small uniform-grid
problems (DFT and 1-D FIO phases, sizes that vary the tree's width product
kappa = N / 2^L), every (r, tol) of a sweep gets an FP64 plan built and
applied on the device, and its relative error (eq:relativeerr) is measured
against the device FP64 direct product.  The network (ibf_mlp_* kernels)
learns log10 of that error; a new problem with accuracy target tol gets the
loosest truncation tolerance (3 tol, tol, tol/3, tol/10), then the smallest
r, whose prediction plus a margin meets tol, with a fixed order as the
fallback.  Every step runs in the library's kernels; this module only
sequences the calls.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import ibf
from . import inputs as I

FALLBACK_R = 12


@dataclass
class TrainingSet:
    X: np.ndarray          # (n, 6) float32 features
    Y: np.ndarray          # (n,) float32 log10 achieved error
    meta: list             # (n, phase, r, tol, err) per sample


HALF_DECADES = tuple(10.0 ** (-e / 2.0) for e in range(5, 19))   # 10^-2.5 .. 10^-9


def generate(ns, phases=(I.PHASE_DFT, I.PHASE_FIO1D), rs=range(3, 15),
             tols=HALF_DECADES, seed: int = 11) -> TrainingSet:
    """Measure the IBF's achieved error over a sweep (FP64 plans, one RHS)."""
    import torch
    ibf.load()
    X, Y, meta = [], [], []
    for n in ns:
        for ph in phases:
            rng = np.random.default_rng(seed + 7919 * n + ph)
            g = I.complex_normal(n, 1, rng)
            x, xi = I.uniform_x(n), I.uniform_xi(n)
            params = I.DEFAULT_PARAMS[ph]
            xd = torch.from_numpy(x).cuda()
            xid = torch.from_numpy(xi).cuda()
            gd = torch.from_numpy(np.ascontiguousarray(g.T)).cuda()
            ud = ibf.dense_apply(ph, params, xd, xid, gd)
            for r in rs:
                for tol in tols:
                    pl = ibf.Plan(x, xi, ph, params, r, tol, 16, I.PREC_FP64, 0).build()
                    u = pl.apply(gd)
                    err, _ = ibf.rel_error(u, ud)          # device FP64 reduction
                    pl.destroy()
                    X.append(ibf.mlp_features(n, ph, r, tol))
                    Y.append(math.log10(max(err, 1e-16)))
                    meta.append((n, ph, r, tol, err))
    return TrainingSet(np.array(X, dtype=np.float32), np.array(Y, dtype=np.float32), meta)


class Predictor:
    """Device-resident parameters of the error model and its Adam state."""

    def __init__(self, n_hidden: int = 16, seed: int = 5, init=None):
        import torch
        self.n_hidden = n_hidden
        npar = ibf.mlp_n_params(n_hidden)
        if init is None:
            init = self.glorot(n_hidden, np.random.default_rng(seed))
        self.params = torch.tensor(np.asarray(init, dtype=np.float32), device="cuda")
        assert self.params.numel() == npar
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    @staticmethod
    def glorot(nh: int, rng: np.random.Generator) -> np.ndarray:
        """Uniform Glorot weights, zero biases, in the flat parameter layout."""
        nf = ibf.MLP_FEATURES
        parts = [rng.uniform(-1, 1, nh * nf) * math.sqrt(6.0 / (nf + nh)), np.zeros(nh),
                 rng.uniform(-1, 1, nh * nh) * math.sqrt(6.0 / (2 * nh)), np.zeros(nh),
                 rng.uniform(-1, 1, nh) * math.sqrt(6.0 / (nh + 1)), np.zeros(1)]
        return np.concatenate(parts)

    def fit(self, data: TrainingSet, steps: int = 6000, lr: float = 1e-2):
        """Full-batch Adam on the mean squared error; returns the final loss."""
        import torch
        X = torch.from_numpy(data.X).cuda()
        T = torch.from_numpy(data.Y).cuda()
        with torch.no_grad():
            self.params[-1] = float(np.mean(data.Y))          # start at the mean target
        loss = None
        for _ in range(steps):
            loss, g = ibf.mlp_loss_grad(self.params, self.n_hidden, X, T)
            self.step += 1
            ibf.mlp_adam(self.params, g, self.m, self.v, self.step, lr)
        torch.cuda.synchronize()
        loss, _ = ibf.mlp_loss_grad(self.params, self.n_hidden, X, T)
        return float(loss.item())

    def predict(self, X: np.ndarray) -> np.ndarray:
        import torch
        y = ibf.mlp_forward(self.params, self.n_hidden,
                            torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda())
        return y.cpu().numpy()

    def select(self, n: int, phase: int, tol: float, margin: float = 0.3):
        """(r, svd_tol) for accuracy target tol, or (FALLBACK_R, tol) when no
        candidate qualifies."""
        r, st = ibf.mlp_select(self.params, self.n_hidden, n, phase, tol, margin)
        return (r, st) if r > 0 else (FALLBACK_R, tol)


def default_sizes():
    """Training sizes: 256..4096 with kappa = N / 2^L spread over (1/2, 1]."""
    return [256, 320, 400, 464, 512, 640, 800, 928, 1024, 1280, 1600, 1856, 2048,
            2560, 3200, 3712, 4096]
