"""GPU parity of the descriptor options against the FP64 oracle, through the
C-ABI: the amplitude a(x, xi) of eqn:FIO (Sec. 1), per-level fixed ranks,
the learned order (r <= 0: the predictor's choice, or the r = 12 fallback),
the automatic sweep-in (Sec. 4.3), and the device relative-error reduction
(eq:relativeerr).  Applied outputs and ranks per level are compared, as in
the main parity tests (FP64 max(1e-12, 8 N 2^-53), FP32 1e-5)."""
import functools
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


def fp64_tol(n):
    return max(1e-12, 8 * n * 2.0 ** -53)


def _apply(torch, pl, g, precision):
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to(dt).cuda()
    u = pl.apply(gt)
    torch.cuda.synchronize()
    return u.cpu().numpy().T.astype(np.complex128)


def _ranks(Op):
    return [v for _, v in sorted(O.level_ranks(Op).items())]


AMPS = {"separable": (O.AMP_SEPARABLE, (1.0, 0.4, -0.3, 1.0, 0.5, 300.0)),
        "wave": (O.AMP_WAVE, (1.0, 0.5, 4096.0))}


@functools.lru_cache(maxsize=None)
def _amp_oracle(name):
    P = I.fio1d_uniform(4096, 10, 3, 41, tol=1e-8)
    amp = AMPS[name]
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf, amp=amp)
    return P, amp, Op, O.apply_optimal(Op, P.g)


@pytest.mark.parametrize("name", ["separable", "wave"])
@pytest.mark.parametrize("precision", [I.PREC_FP64, I.PREC_FP32])
def test_amplitude_parity(torch_dev, name, precision):
    from paper_1605_03616_amd import ibf
    _say(f"amplitude {name} precision={precision}")
    P, amp, Op, u_ref = _amp_oracle(name)
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, precision, amp=amp)
    pl.build()
    u = _apply(torch_dev, pl, P.g, precision)
    q = pl.query()
    pl.destroy()
    tol = fp64_tol(P.n) if precision == I.PREC_FP64 else 1e-5
    assert O.rel_error(u, u_ref) < tol
    assert O.rel_error_cols(u, u_ref) < tol
    assert q["rank"] == _ranks(Op)
    # and the amplitude matters: against the a == 1 operator the gap is O(1)
    u1 = O.dense_apply(P.phase, P.params, P.x, P.xi, P.g[:, :1])
    assert O.rel_error(u[:, :1], u1) > 0.05


def test_fixed_ranks_parity(torch_dev):
    """Caps two below the tolerance ranks at every level: the GPU keeps the
    same per-level ranks as the oracle's capped sweep and the same product."""
    from paper_1605_03616_amd import ibf
    P = I.fio1d_uniform(4096, 10, 2, 42, tol=1e-7)
    prob = O.make_problem(P.phase, P.params, P.x, P.xi, P.r, P.leaf)
    F = O.prelim_factors(prob)
    free = O.level_ranks(O.sweep_out(F, P.tol))
    caps = {l: max(k - 2, 1) for l, k in free.items()}
    Oc = O.sweep_out(F, P.tol, caps=caps)
    u_ref = O.apply_optimal(Oc, P.g)
    caps_arr = [caps[l] for l in sorted(caps)]
    for prec in (I.PREC_FP64, I.PREC_FP32):
        _say(f"fixed ranks {caps_arr} precision={prec}")
        pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, prec,
                      fixed_ranks=caps_arr)
        pl.build()
        u = _apply(torch_dev, pl, P.g, prec)
        q = pl.query()
        pl.destroy()
        assert q["rank"] == _ranks(Oc)
        assert q["nnz_opt"] == O.nnz_optimal(Oc)
        assert O.rel_error(u, u_ref) < (fp64_tol(P.n) if prec == I.PREC_FP64 else 1e-5)


def _step_params(nh=8):
    """A hand-set network in the device layout (hidden width 8, two active
    units): predicted log10 error -6.5 exactly when r >= 8 and the
    truncation tolerance is below 10^-6.5, at least -4.5 otherwise."""
    nf = M.N_FEATURES
    p = np.zeros(M.n_params(nf, nh))
    W1, b1, W2, b2, w3, _ = M.unpack(p, nf, nh)
    K = 1e5
    W1[0, 3], b1[0] = K, -K * 7.5 / 16
    W1[1, 4], b1[1] = K, -K * 6.5 / 16
    W2[0, 0] = W2[1, 1] = 50.0
    w3[:2] = -1.0
    p[-1] = -4.5
    return p, nh


def test_learned_order_from_predictor_and_fallback(torch_dev):
    """r <= 0: with the predictor the build takes the oracle selection's
    (r, truncation) -- (8, 1e-7) for target 1e-6 on the hand-set network --
    and matches the oracle IBF built with them; without a predictor it falls
    back to r = 12 at the target tolerance."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    P = I.fio1d_uniform(2048, 12, 1, 43, tol=1e-6)
    p, nh = _step_params()
    assert M.select(p, nh, P.n, P.phase, P.tol) == (8, 1e-7)
    params = torch.tensor(p.astype(np.float32), device="cuda")
    for pred, (r, st) in [((params, nh), (8, 1e-7)), (None, (12, 1e-6))]:
        _say(f"learned order predictor={'yes' if pred is not None else 'no'}")
        pl = ibf.Plan(P.x, P.xi, P.phase, P.params, 0, P.tol, P.leaf, I.PREC_FP64,
                      predictor=pred)
        pl.build()
        u = _apply(torch, pl, P.g, I.PREC_FP64)
        q = pl.query()
        pl.destroy()
        assert (q["r"], q["learned"]) == (r, 1)
        assert abs(q["tol"] - st) <= 1e-12 * st
        prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, r, st, P.leaf)
        assert q["nnz_prelim"] == O.nnz_prelim(prob)
        assert q["rank"] == _ranks(Op)
        assert O.rel_error(u, O.apply_optimal(Op, P.g)) < fp64_tol(P.n)


def test_sweep_in_auto(torch_dev):
    """sweep_in = -1 with random x and r = 12: some leaf holds fewer than 12
    points, so the sweep-in runs, and the product is the oracle's swept-in
    IBF."""
    from paper_1605_03616_amd import ibf
    P = I.nudft_random(4096, 12, 2, 44, tol=1e-6, precision=I.PREC_FP64, sweep_in=-1)
    _say("sweep-in auto nudft 4096 r=12")
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf)
    Oi = O.sweep_in(Op, P.tol)
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, P.precision, -1)
    pl.build()
    u = _apply(torch_dev, pl, P.g, P.precision)
    q = pl.query()
    pl.destroy()
    assert q["sweep_in"] == 1
    assert O.rel_error(u, O.apply_optimal(Oi, P.g)) < fp64_tol(P.n)


@pytest.mark.parametrize("precision", [I.PREC_FP64, I.PREC_FP32])
def test_device_relative_error(torch_dev, precision):
    """ibf_rel_error against numpy on the same values (ragged columns, one
    column scaled so that the per-column maximum differs from the total)."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    _say(f"rel_error precision={precision}")
    rng = np.random.default_rng(45)
    n, k = 100003, 5
    ref = I.complex_normal(n, k, rng)
    u = ref + 1e-3 * I.complex_normal(n, k, rng)
    u[:, 2] = ref[:, 2] * 1.25
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    ut = torch.from_numpy(np.ascontiguousarray(u.T)).to(dt).cuda()
    rt = torch.from_numpy(np.ascontiguousarray(ref.T)).to(dt).cuda()
    fro, colmax = ibf.rel_error(ut, rt)
    uu = ut.cpu().numpy().T.astype(np.complex128)
    rr = rt.cpu().numpy().T.astype(np.complex128)
    assert abs(fro - O.rel_error(uu, rr)) <= 1e-12 * O.rel_error(uu, rr)
    assert abs(colmax - O.rel_error_cols(uu, rr)) <= 1e-12 * colmax
    assert abs(colmax - 0.25) < 1e-6
