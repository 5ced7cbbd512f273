"""Plain FP64 CPU oracle for the learned Chebyshev-order predictor.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this module; only the tests, the smoke check and the CPU-baseline
leg of the benchmark may.  It shares no code with the HIP implementation.

What is learned.  The paper fixes one Chebyshev order r for the whole
factorization (Sec. 2.1, the interpolation of eqn:ab1 / eqn:ab2) and reports
the achieved relative error (eq:relativeerr) as a function of r, with the
error essentially independent of N (Sec. 6, Tables 1, 3 and 4).  The
predictor is a small multilayer perceptron that models log10 of that
achieved error from problem features, r and the truncation tolerance; for an
accuracy target the plan takes the loosest truncation tolerance, then the
smallest r, whose predicted error, plus a safety margin in decades, meets
the target.  In the collapsed-level geometry every box pair has the same
width product w_A w_B = N / 2^L, so one r serves every level.  The network,
its loss and the Adam optimiser (Kingma and Ba, 2015) are not from the paper.

Network (FP64 here):  h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),
y = w3 . h2 + b3;  loss = mean over samples of (y - target)^2.
Flat parameter layout (an interface shared with the device kernels):
[W1 (H x F, row-major), b1 (H), W2 (H x H, row-major), b2 (H), w3 (H), b3].
"""
from __future__ import annotations

import math

import numpy as np

N_FEATURES = 5
PHASE_DFT, PHASE_FIO1D = 0, 1


def features(n: int, phase: int, r: int, tol: float) -> np.ndarray:
    """x = [kappa, [phase is FIO], [phase is DFT], r/16, -log10(tol)/16] with
    kappa = N / 2^L, L = ceil(log2 N) the tree depth (the width product of
    every box pair in the collapsed-level geometry).  N enters only through
    kappa: the achieved error does not otherwise depend on N (Sec. 6)."""
    L = int(math.ceil(math.log2(n)))
    kappa = n / float(2 ** L)
    return np.array([kappa, 1.0 if phase == PHASE_FIO1D else 0.0,
                     1.0 if phase == PHASE_DFT else 0.0, r / 16.0, -math.log10(tol) / 16.0])


def n_params(nf: int, nh: int) -> int:
    return nh * nf + nh + nh * nh + nh + nh + 1


def unpack(p: np.ndarray, nf: int, nh: int):
    i = 0
    W1 = p[i:i + nh * nf].reshape(nh, nf); i += nh * nf
    b1 = p[i:i + nh]; i += nh
    W2 = p[i:i + nh * nh].reshape(nh, nh); i += nh * nh
    b2 = p[i:i + nh]; i += nh
    w3 = p[i:i + nh]; i += nh
    b3 = p[i]
    return W1, b1, W2, b2, w3, b3


def init_params(nf: int, nh: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform Glorot initialisation of the weights, zero biases."""
    p = np.zeros(n_params(nf, nh))
    W1, b1, W2, b2, w3, b3 = unpack(p, nf, nh)
    W1[...] = rng.uniform(-1, 1, W1.shape) * math.sqrt(6.0 / (nf + nh))
    W2[...] = rng.uniform(-1, 1, W2.shape) * math.sqrt(6.0 / (2 * nh))
    w3[...] = rng.uniform(-1, 1, w3.shape) * math.sqrt(6.0 / (nh + 1))
    return p


def forward(p: np.ndarray, X: np.ndarray, nh: int) -> np.ndarray:
    W1, b1, W2, b2, w3, b3 = unpack(p, X.shape[1], nh)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3


def loss(p: np.ndarray, X: np.ndarray, Y: np.ndarray, nh: int) -> float:
    return float(np.mean((forward(p, X, nh) - Y) ** 2))


def grad(p: np.ndarray, X: np.ndarray, Y: np.ndarray, nh: int) -> np.ndarray:
    """Gradient of the mean squared error by the chain rule, layer by layer."""
    nf = X.shape[1]
    W1, b1, W2, b2, w3, b3 = unpack(p, nf, nh)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ w3 + b3
    dy = 2.0 * (y - Y) / X.shape[0]                 # d loss / d y
    g = np.zeros_like(p)
    gW1, gb1, gW2, gb2, gw3, _ = unpack(g, nf, nh)
    gw3[...] = h2.T @ dy
    g[-1] = dy.sum()
    dz2 = np.outer(dy, w3) * (1.0 - h2 ** 2)        # through tanh'
    gW2[...] = dz2.T @ h1
    gb2[...] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 ** 2)
    gW1[...] = dz1.T @ X
    gb1[...] = dz1.sum(axis=0)
    return g


def adam_step(p, g, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step t >= 1): moment estimates, bias correction,
    per-coordinate step.  Returns the new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(p, X, Y, nh: int, steps: int, lr: float = 1e-2):
    """Full-batch Adam on the mean squared error."""
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in range(1, steps + 1):
        p, m, v = adam_step(p, grad(p, X, Y, nh), m, v, t, lr)
    return p


def select(p, nh: int, n: int, phase: int, tol: float, margin: float = 0.3,
           rmin: int = 2, rmax: int = 16):
    """First (r, svd_tol) whose predicted log10 error + margin <= log10 tol,
    trying the truncation tolerances 3 tol, tol, tol/3, tol/10 (those below 1)
    loosest first and, for each, r ascending; None when none qualifies (the
    caller falls back to a fixed order)."""
    for st in (3.0 * tol, tol, tol / 3.0, tol / 10.0):
        if not st < 1.0:
            continue
        for r in range(rmin, rmax + 1):
            y = forward(p, features(n, phase, r, st)[None, :], nh)[0]
            if y + margin <= math.log10(tol):
                return r, st
    return None
