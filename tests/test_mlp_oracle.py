"""Pins of the FP64 predictor oracle (no GPU): the chain-rule gradient against
central differences and against torch autograd, closed-form forward cases,
the Adam bias-correction identity at t = 1, convergence on a convex
quadratic, and the feature map's tree-depth quantities."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M

NF, NH = M.N_FEATURES, 8


def _data(seed, n=40):
    rng = np.random.default_rng(seed)
    p = M.init_params(NF, NH, rng) + 0.1 * rng.standard_normal(M.n_params(NF, NH))
    X = rng.uniform(-1, 1, (n, NF))
    Y = rng.standard_normal(n)
    return p, X, Y


def test_grad_central_differences():
    p, X, Y = _data(1)
    g = M.grad(p, X, Y, NH)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss(p + e, X, Y, NH) - M.loss(p - e, X, Y, NH)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)


def test_grad_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p, X, Y = _data(2)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    Xt, Yt = torch.tensor(X), torch.tensor(Y)
    i = 0
    W1 = pt[i:i + NH * NF].reshape(NH, NF); i += NH * NF
    b1 = pt[i:i + NH]; i += NH
    W2 = pt[i:i + NH * NH].reshape(NH, NH); i += NH * NH
    b2 = pt[i:i + NH]; i += NH
    w3 = pt[i:i + NH]; i += NH
    b3 = pt[i]
    y = torch.tanh(torch.tanh(Xt @ W1.T + b1) @ W2.T + b2) @ w3 + b3
    torch.mean((y - Yt) ** 2).backward()
    g = M.grad(p, X, Y, NH)
    assert np.allclose(g, pt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_forward_closed_forms():
    rng = np.random.default_rng(3)
    X = rng.uniform(-1, 1, (5, NF))
    p = np.zeros(M.n_params(NF, NH))
    p[-1] = 0.75
    assert np.allclose(M.forward(p, X, NH), 0.75)          # only the output bias
    W1, b1, W2, b2, w3, b3 = M.unpack(p, NF, NH)
    b2[...] = 0.3                                            # W2 = 0: h2 = tanh(b2)
    w3[...] = np.arange(NH)
    want = math.tanh(0.3) * np.arange(NH).sum() + 0.75
    assert np.allclose(M.forward(p, X, NH), want)


def test_adam_first_step_is_sign_step():
    # at t = 1 the bias-corrected moments are g and g^2 exactly, so every
    # coordinate moves by lr * |g| / (|g| + eps) against its gradient
    p, X, Y = _data(4)
    g = M.grad(p, X, Y, NH)
    lr, eps = 1e-3, 1e-8
    p1, _, _ = M.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr, eps=eps)
    step = p - p1
    assert np.allclose(step, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-18)


def test_adam_converges_on_quadratic():
    rng = np.random.default_rng(5)
    target = rng.standard_normal(30)
    scale = rng.uniform(0.5, 5.0, 30)
    p = np.zeros(30)
    m = np.zeros(30)
    v = np.zeros(30)
    for t in range(1, 3001):
        g = 2 * scale * (p - target)
        p, m, v = M.adam_step(p, g, m, v, t, 1e-2)
    assert np.max(np.abs(p - target)) < 1e-3


def test_training_fits_smooth_function():
    rng = np.random.default_rng(6)
    X = rng.uniform(-1, 1, (200, NF))
    Y = np.sin(2 * X[:, 0]) + 0.5 * X[:, 3] ** 2 - X[:, 4]
    p0 = M.init_params(NF, 16, np.random.default_rng(7))
    l0 = M.loss(p0, X, Y, 16)
    p = M.train(p0, X, Y, 16, steps=1500, lr=1e-2)
    assert M.loss(p, X, Y, 16) < 1e-2 * l0


def test_features_tree_quantities():
    f = M.features(4096, M.PHASE_FIO1D, 12, 1e-6)
    assert np.allclose(f, [1.0, 1.0, 0.0, 12 / 16, 6 / 16])
    f = M.features(3000, M.PHASE_DFT, 8, 1e-4)
    assert math.isclose(f[0], 3000 / 4096) and f[1] == 0.0 and f[2] == 1.0
    assert np.allclose(M.features(65536, M.PHASE_DFT, 8, 1e-4), M.features(256, M.PHASE_DFT, 8, 1e-4))
