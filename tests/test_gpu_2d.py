"""2-D multiscale IBF on the GPU against the 2-D oracle (applied outputs and
stored entry counts of the compressed factors), plus the full-size 256 x 256
workload against sampled rows of the dense product.

Bars: FP64 max(1e-12, 8 N 2^-53) relative with N = n^2 points (the phase
evaluation floor: the two libraries' sin / cos / sqrt differ by an ulp and
|Phi| grows with n), FP32 1e-5, BF16X2 1e-4 against the oracle, Frobenius
and per column; the x-independent phase exactly (1e-12).  The 128 x 128
case reaches the 32-wide boxes (three and four stages) of the coronas.
"""
import functools
import os
import sys

import numpy as np
import pytest

from oracle import ibf2d_oracle as D
from oracle import ibf_oracle as O
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
    return float(np.linalg.norm(np.asarray(a, np.complex128) - b) / np.linalg.norm(b))


def fp64_bar(n):
    return max(1e-12, 8 * n * n * 2.0 ** -53)


@pytest.mark.parametrize("phase", [I.PHASE_FIO2D, I.PHASE_DFT, I.PHASE_SEPARABLE])
def test_dense_apply_2d_vs_oracle(torch_dev, phase):
    """The device FP64 direct 2-D product (the dense check bench.py uses)
    against the oracle's, on random x in [0,1)^2 and the integer xi of the
    64 x 64 square: the FP64 phase floor of the grid's size."""
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    _say(f"device dense 2-D product phase={phase}")
    rng = np.random.default_rng(57 + phase)
    n = 64
    x = rng.random((700, 2))
    k = np.arange(n, dtype=np.float64) - n / 2
    xi = np.stack(np.meshgrid(k, k, indexing="ij"), axis=-1).reshape(-1, 2)
    g = I.complex_normal(len(xi), 2, rng)
    params = I.DEFAULT_PARAMS[phase]
    u = ibf.dense_apply_2d(phase, params, torch.from_numpy(x).cuda(),
                           torch.from_numpy(np.ascontiguousarray(xi)).cuda(),
                           torch.from_numpy(np.ascontiguousarray(g.T)).cuda())
    ud = D.dense_apply_2d(phase, params, x, xi, g)
    assert _rel(u.cpu().numpy().T, ud) <= fp64_bar(n)


@functools.lru_cache(maxsize=None)
def _case(n, r, phase=I.PHASE_FIO2D, nrhs=2, seed=41, tol=1e-4):
    P = I.fio2d_grid(n, r, nrhs, seed, tol=tol, precision=I.PREC_FP64)
    P.phase = phase
    P.params = I.DEFAULT_PARAMS[phase]
    part, built, cidx = D.mibf_build(P.phase, P.params, P.x, P.xi, n, r, P.tol)
    u = D.mibf_apply(P.phase, P.params, P.x, P.xi, P.g, built, cidx)
    pre, opt = D.nnz_mibf(built, cidx, len(P.x))
    return P, u, pre, opt


def _gpu(torch, P, precision):
    from paper_1605_03616_amd import ibf
    pl = ibf.Plan.from_problem(P, precision=precision).build()
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(dt).cuda()
    u = pl.apply(g)
    torch.cuda.synchronize()
    q = pl.query()
    pl.destroy()
    return u.cpu().numpy().T.astype(np.complex128), q


@pytest.mark.parametrize("n,r,phase,tol", [(32, 4, I.PHASE_FIO2D, 1e-4),
                                           (64, 5, I.PHASE_FIO2D, 1e-4),
                                           (32, 5, I.PHASE_DFT, 1e-4),
                                           (32, 5, I.PHASE_FIO2D, 1e-9)])
def test_2d_fp64_parity(torch_dev, n, r, phase, tol):
    _say(f"2-D FP64 parity n={n} r={r} phase={phase} tol={tol}")
    P, uo, pre, opt = _case(n, r, phase, tol=tol)
    ug, q = _gpu(torch_dev, P, I.PREC_FP64)
    assert q["nnz_prelim"] == pre
    assert q["nnz_opt"] == opt
    assert _rel(ug, uo) <= fp64_bar(n)
    assert O.rel_error_cols(ug, uo) <= fp64_bar(n)


@pytest.mark.parametrize("precision,bar", [(I.PREC_FP32, 1e-5), (I.PREC_BF16X2, 1e-4)])
def test_2d_reduced_precision(torch_dev, precision, bar):
    _say(f"2-D precision {precision} n=64 r=5")
    P, uo, _, _ = _case(64, 5)
    ug, _ = _gpu(torch_dev, P, precision)
    assert _rel(ug, uo) <= bar
    assert O.rel_error_cols(ug, uo) <= bar


@pytest.mark.parametrize("precision", [I.PREC_FP64, I.PREC_FP32])
def test_2d_128_against_oracle(torch_dev, precision):
    """128 x 128 grid, r = 5, tol 1e-4: the coronas' 32-wide boxes (three H
    and four G stages per box, the batched stage indices 2 and 3) against
    the oracle MIBF, FP64 at its bar and FP32 at 1e-5."""
    _say(f"2-D n=128 r=5 precision={precision}: oracle MIBF (about 30 s)")
    P, uo, pre, opt = _case(128, 5, nrhs=3, seed=44)
    ug, q = _gpu(torch_dev, P, precision)
    bar = fp64_bar(128) if precision == I.PREC_FP64 else 1e-5
    assert _rel(ug, uo) <= bar
    assert O.rel_error_cols(ug, uo) <= bar
    assert q["nnz_prelim"] == pre and q["nnz_opt"] == opt


def test_2d_x_independent_phase_exact(torch_dev):
    _say("2-D separable phase exact")
    P = I.fio2d_grid(32, 3, 1, 42, tol=1e-4, precision=I.PREC_FP64)
    P.phase, P.params = I.PHASE_SEPARABLE, I.DEFAULT_PARAMS[I.PHASE_SEPARABLE]
    ud = D.dense_apply_2d(P.phase, P.params, P.x, P.xi, P.g)
    ug, q = _gpu(torch_dev, P, I.PREC_FP64)
    assert _rel(ug, ud) <= 1e-12
    assert max(q["rank"]) == 1


def test_2d_full_size_fp32(torch_dev):
    """256 x 256 grid, r = 5 x 5, tol 1e-4, 8 RHS FP32 (the benchmark's 2-D
    workload): sampled rows against the dense product (about 1e-2 at r = 5;
    the oracle's factorization at this size is covered by the 128 x 128 case
    above, which has every box width but the 64-wide ring)."""
    P = I.workload_fio2d_256()
    _say("2-D full size 256x256 r=5 FP32 + FP64")
    u32, q32 = _gpu(torch_dev, P, I.PREC_FP32)
    u64, _ = _gpu(torch_dev, P, I.PREC_FP64)
    assert _rel(u32, u64) <= 1e-5
    rows = np.random.default_rng(1234).choice(len(P.x), 256, replace=False)
    ud = D.dense_apply_2d(P.phase, P.params, P.x, P.xi, P.g, rows=rows)
    assert _rel(u32[rows], ud) < 3e-2
    err = _rel(u64[rows], ud)
    _say(f"2-D full size: error vs dense {err:.3g}, R_comp {q32['R_comp']:.3f}")
    assert err < 3e-2
    assert q32["R_comp"] > 1.0


def test_2d_graph_replays_match_direct_launches(torch_dev):
    """The 2-D apply is captured once per (g, u, nrhs, workspace) and replayed:
    every replay, with other GPU work and synchronisations between them, and a
    replay into a new output (a new capture), equals the direct launches
    (IBF_NO_GRAPH) bit for bit; all against the oracle at the FP32 bar."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    _say("2-D graph replay vs direct launches n=64 r=5 FP32")
    P, uo, _, _ = _case(64, 5)
    pl = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
    u = torch.empty((g.shape[0], len(P.x)), dtype=torch.complex64, device="cuda")
    os.environ["IBF_NO_GRAPH"] = "1"
    try:
        pl.apply(g, u)
        torch.cuda.synchronize()
        ref = u.cpu().clone()
    finally:
        del os.environ["IBF_NO_GRAPH"]
    assert _rel(ref.numpy().T, uo) <= 1e-5
    junk = torch.randn(1 << 20, device="cuda")
    for i in range(4):
        u.zero_()
        pl.apply(g, u)
        junk.mul_(1.0001).add_(0.5)                    # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(u.cpu(), ref), f"replay {i}"
    u2 = pl.apply(g)                                   # new output: captured again
    torch.cuda.synchronize()
    assert torch.equal(u2.cpu(), ref)
    pl.destroy()


TABLE4_PARAMS = (2.0, 1.0, 32.0)      # c1, c2 with /32: Table 4's setting (Sec. 6.3)


@functools.lru_cache(maxsize=None)
def _case_high(n, r, tol, table4):
    P = I.fio2d_grid(n, r, 2, 47, tol=tol, precision=I.PREC_FP64)
    if table4:
        P.params = TABLE4_PARAMS
    part, built, cidx = D.mibf_build(P.phase, P.params, P.x, P.xi, n, r, P.tol)
    u = D.mibf_apply(P.phase, P.params, P.x, P.xi, P.g, built, cidx)
    pre, opt = D.nnz_mibf(built, cidx, len(P.x))
    return P, u, pre, opt


@pytest.mark.parametrize("n,r,tol,table4,precision", [
    (32, 6, 1e-3, True, I.PREC_FP64), (32, 6, 1e-3, True, I.PREC_FP32),
    (64, 6, 1e-3, True, I.PREC_FP64), (32, 7, 1e-4, False, I.PREC_FP64),
    (32, 8, 1e-4, False, I.PREC_FP64), (32, 9, 3e-6, True, I.PREC_FP64),
    (32, 9, 3e-6, True, I.PREC_FP32)])
def test_2d_high_order_against_oracle(torch_dev, n, r, tol, table4, precision):
    """r = 6 .. 9 (36 to 81 grid points a box: the compression runs with its
    triangular factor and Jacobi columns in LDS, two rows a lane at r = 9)
    against the oracle MIBF: identical preliminary and stored entry counts,
    FP64 at its bar, FP32 at 1e-5.  r = 6 at tol 1e-3 and r = 9 at 3e-6 with
    c/32 are Table 4's settings: there the GPU factorization also reproduces
    the printed R_comp (within 10 %) and error (within a factor 4, 256
    sampled rows against the dense product)."""
    _say(f"2-D high order n={n} r={r} tol={tol} table4={table4} precision={precision}")
    P, uo, pre, opt = _case_high(n, r, tol, table4)
    ug, q = _gpu(torch_dev, P, precision)
    bar = fp64_bar(n) if precision == I.PREC_FP64 else 1e-5
    assert q["nnz_prelim"] == pre and q["nnz_opt"] == opt
    assert _rel(ug, uo) <= bar
    assert O.rel_error_cols(ug, uo) <= bar
    if table4:
        import json
        golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                             "paper_tables.json")))
        paper = {(row[0], row[1]): (row[2], row[3]) for row in golden["table4_fio2d_mibf"]}
        eps_p, rc_p = paper[(n, r)]
        assert abs(pre / opt / rc_p - 1) < 0.10
        rows = np.random.default_rng(9).choice(len(P.x), 256, replace=False)
        ud = D.dense_apply_2d(P.phase, P.params, P.x, P.xi, P.g[:, :1], rows=rows)
        eps = O.rel_error(ug[rows, :1], ud)
        assert eps_p / 4 < eps < 1.5 * eps_p, (eps, eps_p)


@functools.lru_cache(maxsize=None)
def _case_sampled(n, r, tol, table4, seed, S):
    P = I.fio2d_grid(n, r, 2, 48, tol=tol, precision=I.PREC_FP64)
    if table4:
        P.params = TABLE4_PARAMS
    part, built, cidx = D.mibf_build(P.phase, P.params, P.x, P.xi, n, r, P.tol,
                                     sample=(seed, S))
    u = D.mibf_apply(P.phase, P.params, P.x, P.xi, P.g, built, cidx)
    pre, opt = D.nnz_mibf(built, cidx, len(P.x))
    return P, u, pre, opt


@pytest.mark.parametrize("n,r,tol,table4,S,precision", [
    (32, 5, 1e-4, False, 16, I.PREC_FP64), (32, 9, 3e-6, True, 64, I.PREC_FP64),
    (32, 9, 3e-6, True, 96, I.PREC_FP32), (32, 6, 1e-3, True, 30, I.PREC_FP64)])
def test_2d_sampled_svd_against_oracle(torch_dev, n, r, tol, table4, S, precision):
    """The randomized low-rank approximation (column sampling, svd_samples =
    S) on the register (r = 5) and LDS (r = 6, 9) compression kernels against
    the oracle's sampled factorization with the same seed: identical
    preliminary and stored entry counts (the same columns kept and the same
    ranks), FP64 at its bar, FP32 at 1e-5."""
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    seed = 0x5EED0000 + 17 * r + S
    _say(f"2-D sampled SVD n={n} r={r} tol={tol} S={S} precision={precision}")
    P, uo, pre, opt = _case_sampled(n, r, tol, table4, seed, S)
    pl = ibf.Plan.from_problem(P, precision=precision, svd_sample=(seed, S)).build()
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(dt).cuda()
    ug = pl.apply(g).cpu().numpy().T.astype(np.complex128)
    q = pl.query()
    pl.destroy()
    bar = fp64_bar(n) if precision == I.PREC_FP64 else 1e-5
    assert q["nnz_prelim"] == pre and q["nnz_opt"] == opt
    assert _rel(ug, uo) <= bar
    assert O.rel_error_cols(ug, uo) <= bar
