"""The allocation-free apply (ibf_apply_noalloc) through the C-ABI: the same
product as ibf_apply, bit for bit (same kernels, schedule and summation
order), on two calls in a row that share the static scratch array, the
second with a smaller problem; and the oracle bar on top (FP32 1e-5)."""
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


def _case(torch, P, precision):
    from paper_1605_03616_amd import ibf
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, precision, P.sweep_in)
    pl.build()
    dt = torch.complex128 if precision == I.PREC_FP64 else torch.complex64
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(dt).cuda()
    u_ref = pl.apply(g)
    u = torch.full_like(u_ref, 3.0)
    pl.apply_noalloc(g, u)
    torch.cuda.synchronize()
    return pl, u.cpu().numpy(), u_ref.cpu().numpy()


def test_noalloc_matches_apply_two_calls(torch_dev):
    """A 1-D FIO N = 65536, r = 12, 2-RHS FP32 apply, then a smaller
    random-x N = 4096 problem with the sweep-in in FP64: each equals its
    plan's ibf_apply exactly and the oracle within the bar."""
    torch = torch_dev
    _say("noalloc call 1: fio1d n=65536 r=12 nrhs=2 fp32")
    P1 = I.fio1d_uniform(65536, 12, 2, 51, precision=I.PREC_FP32)
    pl1, u1, r1 = _case(torch, P1, I.PREC_FP32)
    assert np.array_equal(u1, r1)
    _say("noalloc call 2: nudft n=4096 r=10 nrhs=3 fp64 sweep-in")
    P2 = I.nudft_random(4096, 10, 3, 52, precision=I.PREC_FP64, sweep_in=1)
    pl2, u2, r2 = _case(torch, P2, I.PREC_FP64)
    assert np.array_equal(u2, r2)
    prob, F, Op = O.build_optimal(P2.phase, P2.params, P2.x, P2.xi, P2.r, P2.tol, P2.leaf)
    uo = O.apply_optimal(O.sweep_in(Op, P2.tol), P2.g)
    assert O.rel_error(u2.T, uo) < max(1e-12, 8 * P2.n * 2.0 ** -53)
    # the first plan again after the second used the scratch array
    g1 = torch.from_numpy(np.ascontiguousarray(P1.g.T)).to(torch.complex64).cuda()
    u1b = torch.zeros((2, P1.n), dtype=torch.complex64, device="cuda")
    pl1.apply_noalloc(g1, u1b)
    torch.cuda.synchronize()
    assert np.array_equal(u1b.cpu().numpy(), r1)
    pl1.destroy()
    pl2.destroy()


def test_noalloc_rejects_buffers_beyond_the_array(torch_dev):
    """64 RHS at N = 65536 need about 740 MB of coefficient buffers: refused
    with INVALID_ARG before any device work, the output left untouched."""
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    _say("noalloc too large: fio1d n=65536 nrhs=64")
    P = I.fio1d_uniform(65536, 12, 1, 53, precision=I.PREC_FP32)
    pl = ibf.Plan.from_problem(P).build()
    g = torch.zeros((64, P.n), dtype=torch.complex64, device="cuda")
    u = torch.full((64, P.n), 5.0 + 0j, dtype=torch.complex64, device="cuda")
    with pytest.raises(ibf.IBFError) as e:
        pl.apply_noalloc(g, u)
    assert e.value.code == -1 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool(torch.all(u == 5.0).item())
    pl.destroy()
