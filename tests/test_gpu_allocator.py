"""Device memory hook (ibf_set_allocator) with PyTorch's caching allocator:
a 1-D plan, a 2-D plan and a batch take their factors, workspaces and tables
from it (visible in torch.cuda.memory_allocated), applies keep parity with
the FP64 oracle at the FP32 bar, and destroying them returns every block."""
import sys

import numpy as np
import pytest

from oracle import ibf_oracle as O
from paper_1605_03616_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture()
def torch_alloc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1605_03616_amd import ibf
    ibf.load()
    ibf.use_torch_allocator(True)
    try:
        yield torch
    finally:
        ibf.use_torch_allocator(False)


def test_plan_memory_from_torch_allocator(torch_alloc):
    torch = torch_alloc
    from paper_1605_03616_amd import ibf
    _say("allocator hook: fio4k_r12 FP32 plan + batch of two")
    P = I.fio1d_uniform(4096, 12, 8, 25, precision=I.PREC_FP32)
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf,
                                  sweep_in_on=False)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    pl = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    q = pl.query()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base >= q["factor_bytes"]
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
    u = pl.apply(g).cpu().numpy().T.astype(np.complex128)
    assert O.rel_error(u, O.apply_optimal(Op, P.g)) < 1e-5
    # a batch of the plan and a second one: table memory from the hook too
    pl2 = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    b = ibf.Batch([pl, pl2])
    us = b.apply([g, g])
    for ub in us:
        assert O.rel_error(ub.cpu().numpy().T.astype(np.complex128),
                           O.apply_optimal(Op, P.g)) < 1e-5
    del us, u
    b.destroy()
    pl.destroy()
    pl2.destroy()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() - base < 1 << 20      # the vectors g only


def test_2d_plan_memory_from_torch_allocator(torch_alloc):
    torch = torch_alloc
    from paper_1605_03616_amd import ibf
    from oracle import ibf2d_oracle as D
    _say("allocator hook: 2-D n=32 r=4 FP32 plan")
    P = I.fio2d_grid(32, 4, 2, 41, tol=1e-4, precision=I.PREC_FP32)
    part, built, cidx = D.mibf_build(P.phase, P.params, P.x, P.xi, 32, 4, P.tol)
    uo = D.mibf_apply(P.phase, P.params, P.x, P.xi, P.g, built, cidx)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    pl = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() > base
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
    u = pl.apply(g).cpu().numpy().T.astype(np.complex128)
    assert O.rel_error(u, uo) < 1e-5
    pl.destroy()
    del g
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
