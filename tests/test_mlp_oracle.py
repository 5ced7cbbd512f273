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


def _step_network():
    """A hand-set network (2 hidden units) whose output is a step function of
    the features: h1[0] = sign(r - 7.5), h1[1] = sign(-log10(svd_tol) - 6.5)
    (saturated tanh), h2 = sign(h1), y = -4.5 - h2[0] - h2[1].  So y = -6.5
    exactly when r >= 8 and svd_tol < 10^-6.5, and y >= -4.5 otherwise."""
    nf, nh = M.N_FEATURES, 2
    p = np.zeros(M.n_params(nf, nh))
    W1, b1, W2, b2, w3, _ = M.unpack(p, nf, nh)
    K = 1e5
    W1[0, 3], b1[0] = K, -K * 7.5 / 16          # feature 3 is r / 16
    W1[1, 4], b1[1] = K, -K * 6.5 / 16          # feature 4 is -log10(tol) / 16
    W2[0, 0] = W2[1, 1] = 50.0
    w3[:] = -1.0
    p[-1] = -4.5
    return p, nh


def test_select_order_on_a_hand_set_network():
    """The selection tries truncation tolerances 3 tol, tol, tol/3, tol/10
    (those below 1) loosest first and r ascending within each, and returns
    the first whose prediction + margin <= log10 tol: here only
    (r >= 8, svd_tol < 10^-6.5) predicts 10^-6.5, so tol = 1e-6 selects
    (8, 1e-7) -- the first three tolerances (3e-6, 1e-6, 3.3e-7) fail and the
    fourth passes at its smallest qualifying r."""
    p, nh = _step_network()
    y = M.forward(p, np.stack([M.features(1024, 1, r, st) for r in (7, 8)
                               for st in (1e-6, 1e-7)]), nh)
    assert np.allclose(y, [-2.5, -4.5, -4.5, -6.5], atol=1e-12)
    assert M.select(p, nh, 1024, 1, 1e-6) == (8, 1e-7)
    # a target the network never predicts: no candidate (fixed-order fallback)
    assert M.select(p, nh, 1024, 1, 1e-8) is None
    # target 10^-4.4 with margin 0: -4.5 qualifies, so the loosest truncation
    # (3 tol) is kept and r = 8 is the smallest r reaching it
    t = 10.0 ** -4.4
    r, st = M.select(p, nh, 1024, 1, t, margin=0.0)
    assert r == 8 and abs(st - 3 * t) < 1e-18
    # rmin above 8 moves the answer to rmin
    assert M.select(p, nh, 1024, 1, 1e-6, rmin=11) == (11, 1e-7)
    # a target of 0.5: 3 tol = 1.5 is skipped (truncation tolerances stay below 1)
    assert M.select(p, nh, 1024, 1, 0.5, margin=-10.0) == (2, 0.5)
