"""Batched uneven apply (ibf_batch_create / ibf_apply_batch) on the GPU.

Twelve independent 1-D FIO problems with N in [2^10, 2^13] and 1-8 RHS each
(the uneven-batch recipe at reduced sizes).  The batch must reproduce every
plan's own single-plan apply (same kernels and summation order: bitwise, up to
a 1e-6 relative guard), the oracle IBF on every problem (FP32 bar 1e-5,
Frobenius and per column),
and a captured graph must give the eager result on every replay, with other
eager work and synchronisations between the replays.
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


@functools.lru_cache(maxsize=None)
def _batch_problems():
    return I.workload_batched(count=12, seed=3, r=10, lo=10.0, hi=13.0)


@pytest.fixture(scope="module")
def built(torch_dev):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    probs = _batch_problems()
    _say(f"batch build {len(probs)} plans, N={[p.n for p in probs]}")
    plans = [ibf.Plan.from_problem(P) for P in probs]
    for pl in plans:
        pl.build()
    gs = [torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
          for P in probs]
    singles = [pl.apply(g) for pl, g in zip(plans, gs)]
    torch.cuda.synchronize()
    yield probs, plans, gs, [u.cpu().numpy() for u in singles]
    for pl in plans:
        pl.destroy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_batch_matches_single(torch_dev, built):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    probs, plans, gs, ref = built
    _say("batch eager vs single-plan applies")
    B = ibf.Batch(plans)
    us = B.apply(gs, graph=False)
    torch.cuda.synchronize()
    for i, (u, r) in enumerate(zip(us, ref)):
        err = _rel(u.cpu().numpy(), r)
        assert err <= 1e-6, (i, probs[i].n, err)
    B.destroy()


def test_batch_vs_oracle(torch_dev, built):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    probs, plans, gs, _ = built
    B = ibf.Batch(plans)
    us = B.apply(gs, graph=True)
    torch.cuda.synchronize()
    for i, P in enumerate(probs):          # every problem of the batch
        _say(f"batch vs oracle problem {i} N={P.n} nrhs={P.nrhs}")
        _, _, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf,
                                   sweep_in_on=False)
        uo = O.apply_optimal(Op, P.g)
        ug = us[i].cpu().numpy().T.astype(np.complex128)
        assert _rel(ug, uo) <= 1e-5, i
        assert O.rel_error_cols(ug, uo) <= 1e-5, i
    B.destroy()


def test_batch_graph_replays(torch_dev, built):
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    probs, plans, gs, ref = built
    B = ibf.Batch(plans)
    eager = [u.clone() for u in B.apply(gs, graph=False)]
    torch.cuda.synchronize()
    us = [torch.full_like(u, 3.0 + 1.0j) for u in eager]
    for rep in range(3):
        _say(f"batch graph replay {rep}")
        for u in us:
            u.fill_(float(rep) - 2.0j)             # eager work between replays
        B.apply(gs, us, graph=True)
        torch.cuda.synchronize()
        for i, (u, e) in enumerate(zip(us, eager)):
            assert torch.equal(u, e), (rep, i)
        # eager single-plan work in between, then a synchronisation
        plans[rep].apply(gs[rep])
        torch.cuda.synchronize()
    # new output buffers: same graph, table rewritten
    us2 = [torch.zeros_like(u) for u in eager]
    B.apply(gs, us2, graph=True)
    torch.cuda.synchronize()
    for u, e in zip(us2, eager):
        assert torch.equal(u, e)
    B.destroy()


def test_batch_rejects_bad_input(torch_dev, built):
    from paper_1605_03616_amd import ibf
    probs, plans, gs, _ = built
    B = ibf.Batch(plans)
    with pytest.raises(RuntimeError, match="INVALID_ARG"):
        B.apply(gs[:-1] + [gs[0]], graph=False)   # wrong leading dimension for the last plan
    B.destroy()


def test_batch_mixed_installed_schedules(torch_dev):
    """Members with installed schedules in one batch: 16-column MFMA chunks
    for 1 to 8 RHS (some with at most 3 stages a launch) mixed with default
    (vector) members, problems of about 2^14 to 2^15.5 points: eager and
    graph-replayed batches against the single-plan applies with the same
    schedules."""
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    probs = I.workload_batched(count=8, seed=5, r=10, lo=13.5, hi=15.5)
    _say(f"mixed-schedule batch, N={[p.n for p in probs]}")
    plans = [ibf.Plan.from_problem(P).build() for P in probs]
    for i, (pl, P) in enumerate(zip(plans, probs)):
        if i % 3 != 2:
            pl.set_tuning(P.nrhs, "mfma", 16, 3 if i % 2 else 0)
    gs = [torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
          for P in probs]
    ref = [pl.apply(g).cpu().numpy() for pl, g in zip(plans, gs)]
    B = ibf.Batch(plans)
    for graph in (False, True, True):
        us = B.apply(gs, graph=graph)
        torch.cuda.synchronize()
        for i, (u, r) in enumerate(zip(us, ref)):
            err = _rel(u.cpu().numpy(), r)
            assert err <= 1e-6, (graph, i, probs[i].n, err)
    B.destroy()
    for pl in plans:
        pl.destroy()


def test_concurrent_build_matches_sequential(torch_dev, built):
    """ibf_build_batch (worker threads, one stream each) builds the same
    factorizations as one-at-a-time builds: identical ranks, entry counts and
    applied outputs (the builds are deterministic), on 3 worker threads for
    the 12 plans so that each thread builds several."""
    from paper_1605_03616_amd import ibf
    torch = torch_dev
    probs, plans, gs, ref = built
    _say("concurrent build of the batch's plans")
    twins = [ibf.Plan.from_problem(P) for P in probs]
    ibf.build_batch(twins, nthreads=3)
    for i, (a, b) in enumerate(zip(plans, twins)):
        qa, qb = a.query(), b.query()
        assert (qa["rank"], qa["nnz_opt"], qa["nnz_prelim"]) == \
            (qb["rank"], qb["nnz_opt"], qb["nnz_prelim"]), i
    outs = [pl.apply(g) for pl, g in zip(twins, gs)]
    torch.cuda.synchronize()
    for i, (u, r) in enumerate(zip(outs, ref)):
        assert np.array_equal(u.cpu().numpy(), r), i
    # rebuilding some of them again in one call (the previous factors are freed)
    ibf.build_batch(twins[:5], nthreads=8)
    outs = [pl.apply(g) for pl, g in zip(twins[:5], gs[:5])]
    torch.cuda.synchronize()
    for i, (u, r) in enumerate(zip(outs, ref[:5])):
        assert np.array_equal(u.cpu().numpy(), r), i
    for pl in twins:
        pl.destroy()
