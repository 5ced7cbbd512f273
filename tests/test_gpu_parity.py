"""GPU parity: the HIP build + apply (through the C-ABI) against the FP64 oracle.

Applied outputs and per-level ranks are compared (factor entries are not
unique: SVD phases and rotations, zero padding).  Tolerances:
  FP64   max(1e-12, 8 N 2^-53) relative  (the phase-evaluation floor, FP64
         sin/cos of the two libraries differ by an ulp and |Phi| ~ N)
  FP32   1e-5 relative
  BF16X2 1e-4 relative
"""
import functools
import sys

import numpy as np
import pytest

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


def fp64_tol(n):
    return max(1e-12, 8 * n * 2.0 ** -53)


@functools.lru_cache(maxsize=None)
def _oracle(key):
    P = _problems()[key]
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf,
                                  sweep_in_on=False)
    u = O.apply_optimal(Op, P.g)
    return P, prob, Op, u


@functools.lru_cache(maxsize=None)
def _problems():
    return {
        "fio1k_r8": I.workload_fio1d_1k(),
        "dft4k_r10": I.dft_uniform(4096, 10, 3, 21),
        "nudft4k_r10": I.nudft_random(4096, 10, 2, 22, sweep_in=0, precision=I.PREC_FP64),
        "fio3000_r9": I.Problem1D("fio3000", I.uniform_x(3000), I.uniform_xi(3000),
                                  I.PHASE_FIO1D, (2.0, 1.0, 8.0), 9, 1e-6, 16, 2,
                                  I.complex_normal(3000, 2, np.random.default_rng(23)),
                                  I.PREC_FP64),
        "fio256_r6": I.fio1d_uniform(256, 6, 1, 24),
        "fio4k_r12": I.fio1d_uniform(4096, 12, 8, 25, precision=I.PREC_FP32),
        "fio8k_r16": I.fio1d_uniform(8192, 16, 2, 26),
        "fio2k_r2": I.fio1d_uniform(2048, 2, 1, 27, tol=1e-3),
    }


def _run_gpu(torch, P, precision, nrhs=None, ld_pad=0):
    from paper_1605_03616_amd import ibf
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, precision, 0)
    pl.build()
    g = P.g if nrhs is None else P.g[:, :nrhs]
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    nr = g.shape[1]
    gbuf = torch.zeros((nr, P.n + ld_pad), dtype=dt, device="cuda")
    gbuf[:, :P.n] = torch.from_numpy(np.ascontiguousarray(g.T)).to(dt).cuda()
    ubuf = torch.full((nr, P.n + ld_pad), 7.0 + 0j, dtype=dt, device="cuda")
    pl.apply_raw(gbuf.data_ptr(), P.n + ld_pad, ubuf.data_ptr(), P.n + ld_pad, nr)
    torch.cuda.synchronize()
    u = ubuf[:, :P.n].cpu().numpy().T.astype(np.complex128)
    if ld_pad:
        assert torch.all(ubuf[:, P.n:] == 7.0).item()   # padding untouched
    q = pl.query()
    pl.destroy()
    return u, q


def test_kernel_evaluation_matches_definition(torch_dev):
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    rng = np.random.default_rng(40)
    n = 1 << 20
    x = rng.integers(0, n, 20000) / n
    xi = rng.integers(-n // 2, n // 2, 20000).astype(np.float64)
    for kind, prm, tol in [(I.PHASE_DFT, (1.0,), 2e-15), (I.PHASE_DFT, (-1.0,), 2e-15),
                           # c(x) differs by an ulp between the two sine routines and
                           # |xi| <= 2^19 amplifies it: the 8 N 2^-53 floor
                           (I.PHASE_FIO1D, (2.0, 1.0, 8.0), 8 * n * 2.0 ** -53),
                           (I.PHASE_SEPARABLE, (3.0, 0.3125), 2e-15)]:
        _say(f"eval_kernel kind={kind}")
        out = ibf.eval_kernel(kind, prm, torch.from_numpy(x).cuda(),
                              torch.from_numpy(xi).cuda()).cpu().numpy()
        ref = O.kernel(kind, prm, x, xi)
        assert np.max(np.abs(out - ref)) < tol, kind


@pytest.mark.parametrize("key", ["fio1k_r8", "dft4k_r10", "nudft4k_r10", "fio3000_r9",
                                 "fio256_r6", "fio8k_r16", "fio2k_r2"])
def test_fp64_parity(torch_dev, key):
    _say(f"fp64 parity {key}")
    P, prob, Op, u_ref = _oracle(key)
    u, q = _run_gpu(torch_dev, P, I.PREC_FP64)
    err = O.rel_error(u, u_ref)
    assert err < fp64_tol(P.n), (key, err)
    assert O.rel_error_cols(u, u_ref) < fp64_tol(P.n), key
    assert q["rank"] == [v for _, v in sorted(O.level_ranks(Op).items())]
    assert q["nnz_opt"] == O.nnz_optimal(Op)
    assert q["nnz_prelim"] == O.nnz_prelim(prob)


def test_fp64_leading_dimension(torch_dev):
    _say("fp64 ld padding")
    P, prob, Op, u_ref = _oracle("dft4k_r10")
    u, _ = _run_gpu(torch_dev, P, I.PREC_FP64, ld_pad=5)
    assert O.rel_error(u, u_ref) < fp64_tol(P.n)


def test_fp32_parity(torch_dev):
    _say("fp32 parity fio4k_r12")
    P, prob, Op, u_ref = _oracle("fio4k_r12")
    u, q = _run_gpu(torch_dev, P, I.PREC_FP32)
    assert O.rel_error(u, u_ref) < 1e-5
    assert O.rel_error_cols(u, u_ref) < 1e-5
    assert q["rank"] == [v for _, v in sorted(O.level_ranks(Op).items())]


def test_fp32_odd_nrhs_chunks(torch_dev):
    """37 right-hand sides: two RHS chunks, the second partial."""
    _say("fp32 nrhs=37 fio4k_r12")
    P0 = _problems()["fio4k_r12"]
    g = I.complex_normal(P0.n, 37, np.random.default_rng(31))
    P = I.Problem1D("fio4k_r12_37", P0.x, P0.xi, P0.phase, P0.params, P0.r, P0.tol, P0.leaf,
                    37, g, I.PREC_FP32)
    _, prob, Op, _ = _oracle("fio4k_r12")
    u_ref = O.apply_optimal(Op, g)
    u, q = _run_gpu(torch_dev, P, I.PREC_FP32)
    assert O.rel_error(u, u_ref) < 1e-5


def test_fp32_mfma_uneven_leaves(torch_dev):
    """96 right-hand sides on N = 3000: leaves of fewer than 16 points (ragged
    at the end of the grid) through the MFMA leaf products and stages, over
    two 64-column and three 32-column RHS chunks."""
    _say("fp32 nrhs=96 fio3000_r9")
    P0 = _problems()["fio3000_r9"]
    g = I.complex_normal(P0.n, 96, np.random.default_rng(32))
    P = I.Problem1D("fio3000_r9_96", P0.x, P0.xi, P0.phase, P0.params, P0.r, P0.tol, P0.leaf,
                    96, g, I.PREC_FP32)
    _, prob, Op, _ = _oracle("fio3000_r9")
    u_ref = O.apply_optimal(Op, g)
    u, q = _run_gpu(torch_dev, P, I.PREC_FP32)
    assert O.rel_error(u, u_ref) < 1e-5


def test_bf16x2_mfma_parity(torch_dev):
    """BF16x2 factors with 64 right-hand sides: the MFMA kernels widen the
    stored factors to FP32 as they stage them."""
    _say("bf16x2 nrhs=64 fio4k_r12")
    P0 = _problems()["fio4k_r12"]
    g = I.complex_normal(P0.n, 64, np.random.default_rng(33))
    P = I.Problem1D("fio4k_r12_64", P0.x, P0.xi, P0.phase, P0.params, P0.r, P0.tol, P0.leaf,
                    64, g, I.PREC_BF16X2)
    _, prob, Op, _ = _oracle("fio4k_r12")
    u_ref = O.apply_optimal(Op, g)
    u, q = _run_gpu(torch_dev, P, I.PREC_BF16X2)
    assert O.rel_error(u, u_ref) < 1e-4
    assert O.rel_error_cols(u, u_ref) < 1e-4


@pytest.mark.parametrize("key,nrhs,precision,fused,path", [
    ("fio4k_r12", 64, I.PREC_FP32, 0, "tight"), ("fio4k_r12", 130, I.PREC_FP32, 0, "tight"),
    ("fio4k_r12", 64, I.PREC_BF16X2, 0, "tight"), ("fio3000_r9", 70, I.PREC_FP32, 3, "tight"),
    ("fio8k_r16", 64, I.PREC_FP32, 0, "tight"), ("fio2k_r2", 64, I.PREC_FP32, 2, "tight"),
    ("nudft4k_r10", 64, I.PREC_FP32, 0, "tight"), ("fio4k_r12", 64, I.PREC_FP32, 1, "tight"),
    ("nudft4k_r10", 130, I.PREC_FP32, 3, "tight"), ("fio3000_r9", 64, I.PREC_BF16X2, 2, "tight"),
    ("fio4k_r12", 64, I.PREC_BF16X2, 0, "tight_split"),
    ("fio4k_r12", 16, I.PREC_BF16X2, 0, "tight_split"),
    ("fio3000_r9", 70, I.PREC_BF16X2, 3, "tight_split"),
    ("fio8k_r16", 64, I.PREC_BF16X2, 0, "tight_split"),
    ("fio2k_r2", 64, I.PREC_BF16X2, 2, "tight_split"),
    ("nudft4k_r10", 130, I.PREC_BF16X2, 1, "tight_split")])
def test_tight_stage_parity(torch_dev, key, nrhs, precision, fused, path):
    """MFMA stages at each pair's own ranks (64-column chunks, up to 4 stages a
    launch): ragged last chunk (130 = 2 x 64 + 2, 70, 16 of 64 columns live),
    ragged leaves (N = 3000), the widest tile (r = 16), the smallest (r = 2),
    random x, BF16X2 factors widened to FP32 ("tight") and multiplied as BF16
    split products ("tight_split"), and fixed fusion depths (1 to 3 stages a
    launch), against the oracle IBF."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    _say(f"tight stages {key} nrhs={nrhs} precision={precision} fused={fused} path={path}")
    P0 = _problems()[key]
    _, prob, Op, _ = _oracle(key)
    g = I.complex_normal(P0.n, nrhs, np.random.default_rng(36))
    u_ref = O.apply_optimal(Op, g)
    pl = ibf.Plan(P0.x, P0.xi, P0.phase, P0.params, P0.r, P0.tol, P0.leaf, precision, 0)
    pl.build()
    pl.set_tuning(nrhs, path, 0, fused)
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to(torch.complex64).cuda()
    u = pl.apply(gt).cpu().numpy().T.astype(np.complex128)
    prof_u = torch.empty((nrhs, P0.n), dtype=torch.complex64, device="cuda")
    names = {x[0] for x in pl.apply_profile(gt, prof_u)}
    pl.destroy()
    want = "apply_stage_tight_split" if path == "tight_split" else "apply_stage_tight"
    other = "apply_stage_tight" if path == "tight_split" else "apply_stage_tight_split"
    assert want in names and other not in names, names
    tol = 1e-5 if precision == I.PREC_FP32 else 1e-4
    assert O.rel_error(u, u_ref) < tol
    assert O.rel_error_cols(u, u_ref) < tol


def test_bf16x2_parity(torch_dev):
    _say("bf16x2 parity fio4k_r12")
    P, prob, Op, u_ref = _oracle("fio4k_r12")
    u, q = _run_gpu(torch_dev, P, I.PREC_BF16X2)
    assert O.rel_error(u, u_ref) < 1e-4


def test_separable_phase_exact(torch_dev):
    _say("separable exactness")
    P = I.separable_uniform(2048, 4, 2, 30, tol=1e-10)
    u, q = _run_gpu(torch_dev, P, I.PREC_FP64)
    ud = O.dense_apply(P.phase, P.params, P.x, P.xi, P.g)
    assert O.rel_error(u, ud) < 1e-12
    assert all(k == 1 for k in q["rank"])


@pytest.mark.parametrize("key,precision,tol", [
    ("nudft4k_r10", I.PREC_FP64, None),
    ("fio3000_r9", I.PREC_FP64, None),
    ("fio256_r6", I.PREC_FP64, None),
    ("nudft4k_r10", I.PREC_FP32, 1e-5),
])
def test_sweep_in_parity(torch_dev, key, precision, tol):
    """Sweep-in stage (Sec. 4.3) on the GPU against the oracle's sweep-in."""
    _say(f"sweep-in parity {key} precision={precision}")
    P = _problems()[key]
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf)
    Oi = O.sweep_in(Op, P.tol)
    u_ref = O.apply_optimal(Oi, P.g)
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, precision, 1)
    pl.build()
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(dt).cuda()
    u = pl.apply(g).cpu().numpy().T.astype(np.complex128)
    q = pl.query()
    pl.destroy()
    err = O.rel_error(u, u_ref)
    assert err < (fp64_tol(P.n) if tol is None else tol), (key, err)
    T = prob.tree
    assert q["sweep_in"] == 1
    for l, k in Oi.ranks_in["G"].items():
        assert q["rank_in_g"][l - T.l0] == int(np.max(k)), ("G", l)
    for l, k in Oi.ranks_in["H"].items():
        assert q["rank_in_h"][l - T.l0] == int(np.max(k)), ("H", l)
    assert q["nnz_opt"] == O.nnz_optimal_in(Oi)


@functools.lru_cache(maxsize=None)
def _oracle_sweep_in(key):
    P = _problems()[key]
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf)
    return P, O.sweep_in(Op, P.tol)


@pytest.mark.parametrize("nrhs,precision,tol", [(16, I.PREC_BF16X2, 1e-4),
                                                (12, I.PREC_FP32, 1e-5)])
def test_mfma16_sweep_in_parity(torch_dev, nrhs, precision, tol):
    """9 to 16 right-hand sides run the butterfly stages on MFMA in 16-column
    chunks (four slots a wave, up to four fused stages); random x with the
    sweep-in on, as in the non-uniform DFT workload."""
    _say(f"mfma16 sweep-in nudft4k_r10 nrhs={nrhs} precision={precision}")
    P, Oi = _oracle_sweep_in("nudft4k_r10")
    g = I.complex_normal(P.n, nrhs, np.random.default_rng(34))
    u_ref = O.apply_optimal(Oi, g)
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, precision, 1)
    pl.build()
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to(torch.complex64).cuda()
    u = pl.apply(gt).cpu().numpy().T.astype(np.complex128)
    q = pl.query()
    pl.destroy()
    assert q["sweep_in"] == 1
    assert O.rel_error(u, u_ref) < tol


@pytest.mark.parametrize("nrhs,precision", [(20, I.PREC_FP32), (19, I.PREC_FP64),
                                         (33, I.PREC_BF16X2)])
def test_u_leaf_column_chunks(torch_dev, nrhs, precision):
    """16 or more right-hand sides with leaves of more than 16 points (random
    x) run U on the block-per-leaf vector kernel in column chunks (one chunk
    of 19 or 20 columns; 32 + a ragged 1 for 33) against the oracle's
    sweep-in IBF."""
    _say(f"u column chunks nudft4k_r10 nrhs={nrhs} precision={precision}")
    P, Oi = _oracle_sweep_in("nudft4k_r10")
    g = I.complex_normal(P.n, nrhs, np.random.default_rng(35))
    u_ref = O.apply_optimal(Oi, g)
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, precision, 1)
    pl.build()
    assert pl.query()["smax_x"] > 16
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to(dt).cuda()
    u = pl.apply(gt).cpu().numpy().T.astype(np.complex128)
    pl.destroy()
    tol = {I.PREC_FP64: fp64_tol(P.n), I.PREC_FP32: 1e-5, I.PREC_BF16X2: 1e-4}[precision]
    assert O.rel_error(u, u_ref) < tol


def test_determinism(torch_dev):
    _say("run-to-run determinism fio1k")
    P = I.workload_fio1d_1k()
    u1, q1 = _run_gpu(torch_dev, P, I.PREC_FP64)
    u2, q2 = _run_gpu(torch_dev, P, I.PREC_FP64)
    assert np.array_equal(u1, u2) and q1["rank"] == q2["rank"]


def test_full_size_fio64k_fp32(torch_dev):
    """N = 65536, r = 12, 64 RHS, FP32 apply (the benchmark workload, in the
    launch configuration the benchmark times) and the same with BF16X2
    factors (its default schedule: per-pair-rank stages with BF16 split
    products): every column against the oracle's full IBF (Frobenius and
    per-column maximum; FP32 1e-5, BF16X2 1e-4), ranks per level, and the
    dense product on 256 rows."""
    import dataclasses
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    P = I.workload_fio1d_64k(nrhs=64)
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
    res = {}
    for prec in (I.PREC_FP32, I.PREC_BF16X2):
        _say(f"full size fio1d n=65536 r=12 nrhs=64 precision={prec}")
        pl = ibf.Plan.from_problem(dataclasses.replace(P, precision=prec))
        pl.build()
        u = pl.apply(g).cpu().numpy().T.astype(np.complex128)
        prof_u = torch.empty_like(g)
        names = {x[0] for x in pl.apply_profile(g, prof_u)}
        res[prec] = (u, pl.query(), names)
        pl.destroy()
    assert "apply_stage_tight" in res[I.PREC_FP32][2]
    assert "apply_stage_tight_split" in res[I.PREC_BF16X2][2]
    rows = I.error_rows(P.n)
    ud = O.dense_apply(P.phase, P.params, P.x, P.xi, P.g[:, :8], rows=rows)
    assert O.rel_error(res[I.PREC_FP32][0][rows, :8], ud) < 3e-6
    assert O.rel_error(res[I.PREC_BF16X2][0][rows, :8], ud) < 1e-4
    _say("full size fio1d: oracle IBF on all 64 columns")
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf)
    uo = O.apply_optimal(Op, P.g)
    for prec, tol in ((I.PREC_FP32, 1e-5), (I.PREC_BF16X2, 1e-4)):
        u, q, _ = res[prec]
        assert O.rel_error(u, uo) < tol
        assert O.rel_error_cols(u, uo) < tol
        assert q["rank"] == [v for _, v in sorted(O.level_ranks(Op).items())]
        assert q["nnz_opt"] == O.nnz_optimal(Op)


def test_nudft_64k_sweep_in_against_oracle(torch_dev):
    """The random-x workload's distribution at N = 2^16 (x i.i.d. U[0,1) from
    seed 2, r = 10, 16 RHS, sweep-in on): FP32 <= 1e-5 and BF16X2 <= 1e-4
    against the oracle's swept-in IBF, per column too, with the sweep-in
    ranks of both sides equal to the oracle's."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    P = I.workload_nudft_1m(n=1 << 16)
    _say("nudft n=2^16: oracle IBF with sweep-in")
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf)
    Oi = O.sweep_in(Op, P.tol)
    uo = O.apply_optimal(Oi, P.g)
    T = prob.tree
    for prec, tol in [(I.PREC_FP32, 1e-5), (I.PREC_BF16X2, 1e-4)]:
        _say(f"nudft n=2^16 r=10 nrhs=16 sweep-in precision={prec}")
        pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, prec, P.sweep_in)
        pl.build()
        g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
        u = pl.apply(g).cpu().numpy().T.astype(np.complex128)
        q = pl.query()
        pl.destroy()
        assert O.rel_error(u, uo) < tol, prec
        assert O.rel_error_cols(u, uo) < tol, prec
        for l, k in Oi.ranks_in["G"].items():
            assert q["rank_in_g"][l - T.l0] == int(np.max(k)), ("G", l)
        for l, k in Oi.ranks_in["H"].items():
            assert q["rank_in_h"][l - T.l0] == int(np.max(k)), ("H", l)


def test_full_size_nudft_1m_sampled(torch_dev):
    """N = 2^20 random x, r = 10, 16 RHS: BF16X2 and FP32 against the dense
    product on 256 sampled rows, all 16 columns (the oracle IBF at this size
    is covered at 2^16 with the same distribution, above)."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    P = I.workload_nudft_1m()
    rows = I.error_rows(P.n)
    ud = O.dense_apply(P.phase, P.params, P.x, P.xi, P.g, rows=rows)
    for prec, tol in [(I.PREC_FP32, 1e-5), (I.PREC_BF16X2, 1e-4)]:
        _say(f"full size nudft n=2^20 r=10 precision={prec}")
        pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, prec, P.sweep_in)
        pl.build()
        g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
        u = pl.apply(g).cpu().numpy().T.astype(np.complex128)
        pl.destroy()
        assert O.rel_error(u[rows], ud) < tol
        assert O.rel_error_cols(u[rows], ud) < tol
