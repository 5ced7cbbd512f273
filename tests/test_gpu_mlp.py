"""Predictor kernels on the GPU against the FP64 oracle, the device dense
product against the oracle's dense product, and the trained predictor's
gain over the fixed-order fallback (r = 12), checked with the dense oracle:
every chosen (r, truncation) meets its target, the build's
preliminary work shrinks, the stored entries do not grow.

Bars: FP32 gradient and forward against FP64 <= 1e-4 relative; one Adam step
<= 1e-5; dense product max(1e-12, 8 N 2^-53) (the FP64 phase floor); every
selected order must meet its tolerance against the oracle's dense product.
"""
import sys

import numpy as np
import pytest

from oracle import ibf_oracle as O
from oracle import mlp_oracle as M
from paper_1605_03616_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1605_03616_amd import ibf
    ibf.load()
    return torch


def _rel(a, b):
    a = np.asarray(a)
    a = a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("nh", [8, 16, 32])
def test_mlp_forward_and_grad_parity(torch_dev, nh):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    _say(f"mlp forward/grad parity H={nh}")
    rng = np.random.default_rng(100 + nh)
    p = (M.init_params(M.N_FEATURES, nh, rng) + 0.1 * rng.standard_normal(
        M.n_params(M.N_FEATURES, nh))).astype(np.float32)
    X = rng.uniform(-1, 1, (1000, M.N_FEATURES)).astype(np.float32)
    Y = rng.standard_normal(1000).astype(np.float32)
    p64, X64, Y64 = p.astype(np.float64), X.astype(np.float64), Y.astype(np.float64)
    pd, Xd, Yd = (torch.from_numpy(a).cuda() for a in (p, X, Y))
    y = ibf.mlp_forward(pd, nh, Xd).cpu().numpy()
    assert _rel(y, M.forward(p64, X64, nh)) <= 1e-5
    loss, g = ibf.mlp_loss_grad(pd, nh, Xd, Yd)
    assert abs(loss.item() - M.loss(p64, X64, Y64, nh)) <= 1e-5 * M.loss(p64, X64, Y64, nh)
    assert _rel(g.cpu().numpy(), M.grad(p64, X64, Y64, nh)) <= 1e-4


def test_mlp_adam_parity(torch_dev):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    rng = np.random.default_rng(7)
    npar = M.n_params(M.N_FEATURES, 16)
    p, g, m = (rng.standard_normal(npar).astype(np.float32) for _ in range(3))
    v = rng.uniform(0.01, 1.0, npar).astype(np.float32)
    pd, gd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (p, g, m, v))
    ibf.mlp_adam(pd, gd, md, vd, 7, 1e-2)
    p2, m2, v2 = M.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                             v.astype(np.float64), 7, 1e-2)
    assert _rel(pd.cpu().numpy(), p2) <= 1e-5
    assert _rel(md.cpu().numpy(), m2) <= 1e-5 and _rel(vd.cpu().numpy(), v2) <= 1e-5


def test_mlp_features_match_oracle(torch_dev):
    from paper_1605_03616_amd import ibf
    for n, ph, r, tol in [(256, 1, 8, 1e-6), (3000, 0, 11, 1e-4), (65482, 1, 12, 1e-6)]:
        assert np.allclose(ibf.mlp_features(n, ph, r, tol), M.features(n, ph, r, tol),
                           rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("phase", [I.PHASE_DFT, I.PHASE_FIO1D])
def test_dense_apply_vs_oracle(torch_dev, phase):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    n = 1500
    _say(f"device dense product phase={phase} N={n}")
    rng = np.random.default_rng(31 + phase)
    x = rng.random(n)
    xi = I.uniform_xi(n)
    g = I.complex_normal(n, 2, rng)
    params = I.DEFAULT_PARAMS[phase]
    u = ibf.dense_apply(phase, params, torch.from_numpy(x).cuda(), torch.from_numpy(xi).cuda(),
                        torch.from_numpy(np.ascontiguousarray(g.T)).cuda())
    ud = O.dense_apply(phase, params, x, xi, g)
    assert _rel(u.cpu().numpy().T, ud) <= max(1e-12, 8 * n * 2.0 ** -53)


def test_predictor_trains_and_gains(torch_dev):
    from paper_1605_03616_amd import ibf
    from paper_1605_03616_amd import predictor as PR
    torch = torch_dev
    _say("predictor: training data on the device")
    data = PR.generate([256, 400, 640, 1024, 1600])
    _say(f"predictor: {len(data.Y)} samples, training")
    pred = PR.Predictor(n_hidden=16, seed=5)
    final = pred.fit(data, steps=6000, lr=1e-2)
    rmse = float(np.sqrt(np.mean((pred.predict(data.X) - data.Y) ** 2)))
    _say(f"predictor: training loss {final:.4g}, rmse {rmse:.3f} decades")
    assert rmse <= 0.2
    # held-out sizes and targets, each choice checked against the oracle's dense product.
    # The gain: the stored (apply) entries follow the truncation tolerance and
    # stay the same, while the build's work (preliminary entries ~ r^2 per
    # pair and level, SVDs of r x 2r blocks) shrinks with the smaller order.
    tot = {"pre_p": 0, "pre_f": 0, "opt_p": 0, "opt_f": 0, "ms_p": 0.0, "ms_f": 0.0}
    smaller = 0
    cases = [(1300, I.PHASE_FIO1D, 1e-4), (2000, I.PHASE_FIO1D, 1e-6),
             (1300, I.PHASE_DFT, 1e-6), (2000, I.PHASE_DFT, 1e-4)]
    for n, ph, tol in cases:
        r, st = pred.select(n, ph, tol)
        _say(f"predictor: N={n} phase={ph} target={tol:g} -> r={r}, truncation {st:g}")
        x, xi = I.uniform_x(n), I.uniform_xi(n)
        g = I.complex_normal(n, 1, np.random.default_rng(n + ph))
        ud = O.dense_apply(ph, I.DEFAULT_PARAMS[ph], x, xi, g)
        gd = torch.from_numpy(np.ascontiguousarray(g.T)).cuda()
        res = {}
        for key, (rr, tt) in (("p", (r, st)), ("f", (PR.FALLBACK_R, tol))):
            pl = ibf.Plan(x, xi, ph, I.DEFAULT_PARAMS[ph], rr, tt, 16, I.PREC_FP64, 0).build()
            q = pl.query()
            res[key] = _rel(pl.apply(gd).cpu().numpy().T, ud)
            tot["pre_" + key] += q["nnz_prelim"]
            tot["opt_" + key] += q["nnz_opt"]
            tot["ms_" + key] += q["build_ms"]
            pl.destroy()
        _say(f"predictor:   error {res['p']:.3g} (fixed r={PR.FALLBACK_R}: {res['f']:.3g})")
        assert res["p"] <= tol, (n, ph, tol, r, st, res["p"])
        smaller += r < PR.FALLBACK_R
    _say(f"predictor: preliminary entries {tot['pre_p'] / tot['pre_f']:.3f}x, stored entries "
         f"{tot['opt_p'] / tot['opt_f']:.3f}x, build ms {tot['ms_p']:.1f} vs {tot['ms_f']:.1f}, "
         f"smaller r in {smaller}/{len(cases)}")
    assert smaller >= 3
    assert tot["pre_p"] < 0.8 * tot["pre_f"]
    assert tot["opt_p"] <= 1.05 * tot["opt_f"]
