"""Host-side checks of the C-ABI: the library loads, exports every symbol
that include/ibf.h declares, and validates descriptors without touching a
device (ibf_plan is host-only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import ibf_oracle as O
from paper_1605_03616_amd import ibf
from paper_1605_03616_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "ibf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\*)\s+(ibf_\w+)\s*\(", src, re.M)))


def test_header_and_binding_agree():
    decl = _declared_symbols()
    assert decl == sorted(ibf.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ibf.load()
    for name in _declared_symbols():
        assert hasattr(lib, name), name


def _plan(**kw):
    P = I.workload_fio1d_1k()
    args = dict(x=P.x, xi=P.xi, phase=P.phase, params=P.params, r=P.r, tol=P.tol,
                leaf=P.leaf, precision=P.precision)
    args.update(kw)
    return ibf.Plan(**args)


def test_plan_and_query_geometry():
    pl = _plan()
    q = pl.query()
    assert (q["L"], q["l0"], q["h"], q["n_levels"]) == (10, 4, 5, 3)
    assert q["n_pairs"] == 1024
    assert q["smax_x"] == 16 and q["smax_xi"] == 16
    # the oracle's count, itself recounted from the explicit sparse factors
    P = I.workload_fio1d_1k()
    assert q["nnz_prelim"] == O.nnz_prelim(O.make_problem(P.phase, P.params, P.x, P.xi, P.r, P.leaf))
    assert (q["r"], q["learned"], q["sweep_in"]) == (8, 0, 0)
    pl.destroy()


def test_plan_geometry_ragged_and_odd_depth():
    P = I.nudft_random(2048, 6, 1, 7)
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, 6, 1e-6, 16, I.PREC_FP32)
    q = pl.query()
    assert (q["L"], q["l0"], q["h"]) == (11, 4, 5)
    cnt = np.bincount(np.floor(P.x * 128).astype(int), minlength=128)
    assert q["smax_x"] == cnt.max()
    pl.destroy()


@pytest.mark.parametrize("kw,code", [
    (dict(r=1), "INVALID_ARG"),
    (dict(r=17), "UNSUPPORTED"),
    (dict(tol=0.0), "INVALID_ARG"),
    (dict(tol=1.5), "INVALID_ARG"),
    (dict(leaf=12), "INVALID_ARG"),
    (dict(leaf=64), "INVALID_ARG"),          # 1024 < 64^2
    (dict(precision=7), "INVALID_ARG"),
    (dict(phase=9), "UNSUPPORTED"),
    (dict(x=np.full(1024, 1.0)), "INVALID_ARG"),   # outside [0,1)
    (dict(xi=np.arange(1024.0) + 600), "INVALID_ARG"),
])
def test_plan_rejects_bad_descriptors(kw, code):
    with pytest.raises(ibf.IBFError) as ei:
        _plan(**kw)
    assert code in str(ei.value)


def test_apply_before_build_is_not_built():
    pl = _plan()
    lib = ibf.load()
    rc = lib.ibf_apply(pl.handle, C.c_void_p(1), 1024, C.c_void_p(2), 1024, 1, None)
    assert rc == -5
    assert "not built" in ibf.last_error()
    pl.destroy()


def test_adjoint_validates_before_device_work():
    lib = ibf.load()
    assert lib.ibf_apply_adjoint(None, C.c_void_p(1), 1024, C.c_void_p(2), 1024, 1, None) == -1
    pl = _plan()
    rc = lib.ibf_apply_adjoint(pl.handle, C.c_void_p(1), 1024, C.c_void_p(2), 1024, 1, None)
    assert rc == -5                                  # not built
    assert "not built" in ibf.last_error()
    pl.destroy()


def test_null_arguments():
    lib = ibf.load()
    assert lib.ibf_plan(None, None) == -1
    assert lib.ibf_build(None, None) == -1
    assert lib.ibf_query(None, None) == -1
    assert lib.ibf_destroy(None) == 0


def test_set_tuning_validates_host_only():
    # installing a schedule touches no device: checked on an unbuilt plan
    lib = ibf.load()
    pl = _plan(precision=I.PREC_FP32)
    T = ibf.IBFTuning
    assert lib.ibf_set_tuning(None, 8, C.byref(T(0, 0, 0, 0.0))) == -1
    assert lib.ibf_set_tuning(pl.handle, 0, C.byref(T(0, 0, 0, 0.0))) == -1
    for bad in [T(5, 0, 0, 0.0), T(-1, 0, 0, 0.0), T(2, 8, 0, 0.0), T(1, 0, -1, 0.0),
                T(0, 0, 0, 0.0, 3)]:
        assert lib.ibf_set_tuning(pl.handle, 8, C.byref(bad)) == -1
    assert lib.ibf_set_tuning(pl.handle, 8, C.byref(T(2, 32, 3, 0.0))) == 0
    assert lib.ibf_set_tuning(pl.handle, 8, None) == 0          # back to the default rule
    pl.set_tuning(12, "vector", 0, 2)
    pl.set_tuning(12, "mfma", 16, 0, 2)
    pl.set_tuning(64, "tight", 0, 3)
    pl.set_tuning(12)
    # BF16 split products (path 4) need BF16X2 factors
    assert lib.ibf_set_tuning(pl.handle, 64, C.byref(T(4, 0, 0, 0.0))) == -2
    pl.destroy()
    pbf = _plan(precision=I.PREC_BF16X2)
    pbf.set_tuning(64, "tight_split", 0, 2)
    pbf.set_tuning(64, "tight", 0, 0)
    pbf.destroy()
    p64 = _plan(precision=I.PREC_FP64)
    assert lib.ibf_set_tuning(p64.handle, 8, C.byref(T(2, 16, 0, 0.0))) == -2
    assert lib.ibf_set_tuning(p64.handle, 8, C.byref(T(3, 0, 0, 0.0))) == -2
    assert lib.ibf_set_tuning(p64.handle, 8, C.byref(T(4, 0, 0, 0.0))) == -2
    assert lib.ibf_set_tuning(p64.handle, 8, C.byref(T(1, 0, 2, 0.0))) == 0
    p64.destroy()


def test_set_allocator_arguments():
    # host only: installs or clears the hook, no device call
    lib = ibf.load()
    a = ibf.ALLOC_FN(lambda n, s: None)
    assert lib.ibf_set_allocator(a, ibf.FREE_FN()) == -1          # one of the two
    assert lib.ibf_set_allocator(ibf.ALLOC_FN(), ibf.FREE_FN()) == 0


def test_mlp_feature_map_matches_oracle():
    # host-only entry point: the predictor's features against the oracle's
    from oracle import mlp_oracle as M
    for n, ph, r, tol in [(256, 1, 8, 1e-6), (3000, 0, 11, 1e-4), (65482, 1, 12, 1e-6),
                          (1025, 3, 5, 0.5)]:
        assert np.allclose(ibf.mlp_features(n, ph, r, tol), M.features(n, ph, r, tol),
                           rtol=1e-6, atol=1e-7)
    for h in (8, 16, 32):
        assert ibf.mlp_n_params(h) == M.n_params(M.N_FEATURES, h)
    with pytest.raises(ValueError):
        ibf.mlp_n_params(12)
    with pytest.raises(ibf.IBFError):
        ibf.mlp_features(1024, 1, 8, 0.0)


def test_sweep_in_auto_follows_leaf_populations():
    """sweep_in = -1 turns the sweep-in on iff a leaf holds fewer than r points
    (Sec. 4.3): off on the uniform grid (every leaf full), on for random x
    with r = 12 (Poisson(16) leaves), off again there at r = 4."""
    pl = _plan(sweep_in=-1)
    assert pl.query()["sweep_in"] == 0
    pl.destroy()
    P = I.nudft_random(4096, 12, 1, 2)
    cnt = np.bincount(np.floor(P.x * 256).astype(int), minlength=256)
    for r in (12, 4):
        pl = ibf.Plan(P.x, P.xi, P.phase, P.params, r, 1e-6, 16, I.PREC_FP32, sweep_in=-1)
        assert pl.query()["sweep_in"] == int(cnt.min() < r), (r, cnt.min())
        pl.destroy()
    assert cnt.min() < 12 and cnt.min() >= 4


def test_learned_order_plan_defers_r_to_the_build():
    """r <= 0: the plan is valid, the order is chosen at build time."""
    pl = _plan(r=0)
    q = pl.query()
    assert (q["r"], q["learned"], q["nnz_prelim"]) == (0, 1, 0)
    pl.destroy()
    with pytest.raises(ibf.IBFError) as e:
        _plan(r=0, predictor=(_FakeTensor(), 7))
    assert e.value.code == -1


class _FakeTensor:
    def __init__(self):
        self.buf = np.zeros(4, dtype=np.float32)

    def data_ptr(self):
        return self.buf.ctypes.data


@pytest.mark.parametrize("amp,code", [((1, (1.0, 0.5, 0.0, 1.0, 0.5)), -1),     # 5 of 6 params
                                      ((1, (1.0, 0.5, 0.0, 1.0, 0.5, 0.0)), -1),  # q5 == 0
                                      ((2, (1.0, 0.5, 0.0)), -1),                 # q2 == 0
                                      ((7, (1.0,)), -2)])                          # unknown
def test_amplitude_descriptor_validation(amp, code):
    with pytest.raises(ibf.IBFError) as e:
        _plan(amp=amp)
    assert e.value.code == code


def test_amplitude_and_caps_rejected_for_dim2():
    n = 32
    i1, i2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = np.stack([i1.ravel() / n, i2.ravel() / n], -1)
    xi = np.stack([i1.ravel() - n // 2, i2.ravel() - n // 2], -1).astype(np.float64)
    for kw in (dict(amp=(2, (1.0, 0.5, 64.0))), dict(fixed_ranks=[3] * 8)):
        with pytest.raises(ibf.IBFError) as e:
            ibf.Plan(x, xi, 2, (2.0, 1.0, 16.0), 5, 1e-4, 16, I.PREC_FP32, **kw)
        assert e.value.code == -2
    # orders 2 .. 9 (up to 81 tensor grid points a box)
    for r, code in ((9, 0), (10, -2), (1, -1)):
        if code == 0:
            ibf.Plan(x, xi, 2, (2.0, 1.0, 16.0), r, 1e-4, 16, I.PREC_FP32).destroy()
            continue
        with pytest.raises(ibf.IBFError) as e:
            ibf.Plan(x, xi, 2, (2.0, 1.0, 16.0), r, 1e-4, 16, I.PREC_FP32)
        assert e.value.code == code


def test_rel_error_validates_on_the_host():
    lib = ibf.load()
    out = (C.c_double * 2)()
    assert lib.ibf_rel_error(None, 4, None, 4, 4, 1, 0, out, None) == -1
    buf = np.zeros(8)
    ptr = C.c_void_p(buf.ctypes.data)
    assert lib.ibf_rel_error(ptr, 2, ptr, 4, 4, 1, 0, out, None) == -1     # ldu < n
    assert lib.ibf_rel_error(ptr, 4, ptr, 4, 4, 0, 0, out, None) == -1     # nrhs < 1


def test_build_batch_validates_on_the_host():
    """ibf_build_batch rejects bad plan lists before any device call."""
    lib = ibf.load()
    pl = _plan()
    failed = C.c_int(7)
    twice = (C.c_void_p * 2)(pl.handle, pl.handle)
    assert lib.ibf_build_batch(twice, 2, 0, None, C.byref(failed)) == -1
    assert failed.value == -1 and "twice" in ibf.last_error()
    assert lib.ibf_build_batch(twice, 0, 0, None, None) == -1
    assert lib.ibf_build_batch(None, 2, 0, None, None) == -1
    holes = (C.c_void_p * 2)(pl.handle, None)
    assert lib.ibf_build_batch(holes, 2, 0, None, None) == -1
    pl.destroy()


def test_sampled_svd_descriptor_validation():
    """svd_samples: negative is INVALID_ARG; the 1-D plans (blocks of at most
    32 columns) leave the sampled approximation out: UNSUPPORTED; dim 2
    accepts it on the host."""
    with pytest.raises(ibf.IBFError) as e:
        _plan(svd_sample=(1, -3))
    assert e.value.code == -1
    with pytest.raises(ibf.IBFError) as e:
        _plan(svd_sample=(1, 16))
    assert e.value.code == -2
    n = 32
    i1, i2 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    x = np.stack([i1.ravel() / n, i2.ravel() / n], -1)
    xi = np.stack([i1.ravel() - n // 2, i2.ravel() - n // 2], -1).astype(np.float64)
    ibf.Plan(x, xi, 2, (2.0, 1.0, 16.0), 6, 1e-3, 16, I.PREC_FP32, svd_sample=(7, 24)).destroy()
    with pytest.raises(ibf.IBFError) as e:
        ibf.Plan(x, xi, 2, (2.0, 1.0, 16.0), 6, 1e-3, 16, I.PREC_FP32, svd_sample=(7, -1))
    assert e.value.code == -1


def test_dense_apply_arguments_host_only():
    # argument and phase checks happen before any device call
    lib = ibf.load()
    vp = C.c_void_p(16)                                      # never dereferenced
    for fn in (lib.ibf_dense_apply, lib.ibf_dense_apply_2d):
        assert fn(I.PHASE_DFT, None, 0, None, 4, vp, 4, vp, 4, vp, 4, 1, None) == -1
        assert fn(I.PHASE_DFT, None, 0, vp, 4, vp, 4, vp, 3, vp, 4, 1, None) == -1   # ldg < n_xi
        assert fn(I.PHASE_DFT, None, 0, vp, 4, vp, 4, vp, 4, vp, 4, 0, None) == -1   # nrhs < 1
        assert fn(I.PHASE_DFT, None, -1, vp, 4, vp, 4, vp, 4, vp, 4, 1, None) == -1
        assert fn(7, None, 0, vp, 4, vp, 4, vp, 4, vp, 4, 1, None) == -2
    # each dimension refuses the other's phase
    assert lib.ibf_dense_apply(I.PHASE_FIO2D, None, 0, vp, 4, vp, 4, vp, 4, vp, 4, 1, None) == -2
    assert lib.ibf_dense_apply_2d(I.PHASE_FIO1D, None, 0, vp, 4, vp, 4, vp, 4, vp, 4, 1,
                                  None) == -2
    bad = (C.c_double * 3)(2.0, 1.0, 0.0)                    # FIO2D with p2 == 0
    assert lib.ibf_dense_apply_2d(I.PHASE_FIO2D, bad, 3, vp, 4, vp, 4, vp, 4, vp, 4, 1,
                                  None) == -1
    # nothing to do: no device call
    assert lib.ibf_dense_apply_2d(I.PHASE_FIO2D, None, 0, vp, 0, vp, 4, vp, 4, vp, 4, 1,
                                  None) == 0
