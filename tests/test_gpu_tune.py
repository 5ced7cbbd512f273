"""Schedule autotuner (ibf_tune): it picks one of its candidates, never one
slower than the default rule it also times, and the applies that follow keep
parity with the FP64 oracle (every candidate computes the same product: the
stages of the paper's factorization, Sec. 4, grouped differently into
launches).  FP32 bar 1e-5 relative, as for every FP32 apply."""
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


@functools.lru_cache(maxsize=None)
def _oracle():
    P = I.fio1d_uniform(4096, 12, 8, 25, precision=I.PREC_FP32)
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf,
                                  sweep_in_on=False)
    return P, Op


@pytest.mark.parametrize("nrhs", [8, 37])
def test_tune_then_apply_parity(torch_dev, nrhs):
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    _say(f"tune fio4k_r12 nrhs={nrhs}")
    P, Op = _oracle()
    g = I.complex_normal(P.n, nrhs, np.random.default_rng(40 + nrhs))
    u_ref = O.apply_optimal(Op, g)
    pl = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to(torch.complex64).cuda()
    res = pl.tune(gt)
    torch.cuda.synchronize()
    assert res["path"] in ("default", "vector", "mfma", "tight")
    assert res["ms"] > 0 and res["default_ms"] > 0
    assert res["ms"] <= res["default_ms"] * (1 + 1e-6)       # the default is a candidate
    u = pl.apply(gt).cpu().numpy().T.astype(np.complex128)   # with the tuned schedule
    pl.destroy()
    assert O.rel_error(u, u_ref) < 1e-5, res


@pytest.mark.parametrize("sched", [("vector", 0, 2), ("mfma", 16, 3), ("mfma", 32, 2),
                                   ("mfma", 16, 0), ("mfma", 16, 0, 1), ("mfma", 32, 0, 2),
                                   ("default", 0, 0, 2), ("tight", 0, 0), ("tight", 0, 3),
                                   ("tight", 0, 1)])
def test_fixed_schedule_parity(torch_dev, sched):
    # ibf_set_tuning installs a schedule without timing: same product
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    nrhs = 37
    _say(f"fixed schedule {sched} fio4k_r12 nrhs={nrhs}")
    P, Op = _oracle()
    g = I.complex_normal(P.n, nrhs, np.random.default_rng(77))
    u_ref = O.apply_optimal(Op, g)
    pl = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    pl.set_tuning(nrhs, *sched)
    gt = torch.from_numpy(np.ascontiguousarray(g.T)).to(torch.complex64).cuda()
    u = pl.apply(gt).cpu().numpy().T.astype(np.complex128)
    pl.set_tuning(nrhs)                                       # default rule again
    u0 = pl.apply(gt).cpu().numpy().T.astype(np.complex128)
    pl.destroy()
    assert O.rel_error(u, u_ref) < 1e-5
    assert O.rel_error(u0, u_ref) < 1e-5


def test_tune_2d_unsupported(torch_dev):
    torch = torch_dev
    from paper_1605_03616_amd import ibf
    _say("tune 2-D plan: unsupported")
    P = I.fio2d_grid(32, 3, 1, 42, tol=1e-4, precision=I.PREC_FP32)
    pl = ibf.Plan.from_problem(P, precision=I.PREC_FP32).build()
    gt = torch.zeros((1, len(P.xi)), dtype=torch.complex64, device="cuda")
    with pytest.raises(ibf.IBFError) as err:
        pl.tune(gt)
    assert err.value.code == -2                               # IBF_ERR_UNSUPPORTED
    pl.destroy()
