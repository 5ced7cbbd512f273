"""Thin ctypes binding of libibf.so (the C-ABI in include/ibf.h).

Argument marshalling only: every step of the factorization and of its
application runs in the library's HIP kernels.  PyTorch supplies device
memory and the current stream.  If the library is missing this module
raises at import of the library, never falls back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .inputs import PREC_BF16X2, PREC_FP32, PREC_FP64  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibf.so")

IBF_OK = 0
ERRORS = {-1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "OOM", -4: "DEVICE", -5: "NOT_BUILT"}

EXPORTED = ["ibf_plan", "ibf_build", "ibf_apply", "ibf_apply_profile", "ibf_query",
            "ibf_destroy", "ibf_last_error", "ibf_eval_kernel", "ibf_batch_create",
            "ibf_apply_batch", "ibf_batch_destroy", "ibf_dense_apply", "ibf_mlp_n_params",
            "ibf_mlp_features", "ibf_mlp_forward", "ibf_mlp_grad_work", "ibf_mlp_loss_grad",
            "ibf_mlp_adam", "ibf_mlp_select", "ibf_tune", "ibf_set_tuning", "ibf_set_allocator",
            "ibf_measure_peak", "ibf_apply_adjoint", "ibf_rel_error", "ibf_apply_noalloc",
            "ibf_build_batch", "ibf_dense_apply_2d"]
MLP_FEATURES = 5
PATHS = ["default", "vector", "mfma", "tight", "tight_split"]      # ibf_tuning.path
BATCH_GRAPH = 1
PROFILE_MAX = 64


class IBFDesc(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n_x", C.c_int64),
        ("n_xi", C.c_int64),
        ("x", C.POINTER(C.c_double)),
        ("xi", C.POINTER(C.c_double)),
        ("omega_lo", C.c_double),
        ("omega_width", C.c_double),
        ("phase_id", C.c_int),
        ("phase_params", C.POINTER(C.c_double)),
        ("n_params", C.c_int),
        ("r", C.c_int),
        ("tol", C.c_double),
        ("leaf", C.c_int),
        ("precision", C.c_int),
        ("sweep_in", C.c_int),
        ("device", C.c_int),
        ("fixed_ranks", C.POINTER(C.c_int)),
        ("amp_id", C.c_int),
        ("amp_params", C.POINTER(C.c_double)),
        ("n_amp_params", C.c_int),
        ("predictor", C.c_void_p),
        ("predictor_hidden", C.c_int),
        ("svd_samples", C.c_int),
        ("svd_seed", C.c_uint64),
    ]


class IBFInfo(C.Structure):
    _fields_ = [
        ("L", C.c_int), ("l0", C.c_int), ("h", C.c_int), ("n_levels", C.c_int),
        ("rank", C.c_int * 64),
        ("n_pairs", C.c_int64),
        ("nnz_prelim", C.c_int64),
        ("nnz_opt", C.c_int64),
        ("nnz_stored", C.c_int64),
        ("factor_bytes", C.c_int64),
        ("build_ms", C.c_double),
        ("smax_x", C.c_int), ("smax_xi", C.c_int),
        ("sweep_in", C.c_int),
        ("rank_in_g", C.c_int * 64),
        ("rank_in_h", C.c_int * 64),
        ("r", C.c_int),
        ("tol", C.c_double),
        ("learned", C.c_int),
    ]


class IBFTuning(C.Structure):
    _fields_ = [("path", C.c_int), ("chunk", C.c_int), ("max_fused", C.c_int), ("ms", C.c_float),
                ("split", C.c_int)]


class IBFProfile(C.Structure):
    _fields_ = [
        ("n_launches", C.c_int),
        ("name", (C.c_char * 24) * PROFILE_MAX),
        ("ms", C.c_float * PROFILE_MAX),
        ("flops", C.c_double * PROFILE_MAX),
        ("bytes", C.c_double * PROFILE_MAX),
        ("vec_bytes", C.c_double * PROFILE_MAX),
    ]


class IBFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libibf.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with paper_1605_03616_amd.build_lib")
    lib = C.CDLL(path)
    lib.ibf_plan.argtypes = [C.POINTER(IBFDesc), C.POINTER(C.c_void_p)]
    lib.ibf_build.argtypes = [C.c_void_p, C.c_void_p]
    lib.ibf_apply.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                              C.c_int64, C.c_void_p]
    lib.ibf_apply_profile.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                      C.c_int64, C.c_int64, C.c_void_p, C.POINTER(IBFProfile)]
    lib.ibf_query.argtypes = [C.c_void_p, C.POINTER(IBFInfo)]
    lib.ibf_destroy.argtypes = [C.c_void_p]
    lib.ibf_last_error.restype = C.c_char_p
    lib.ibf_eval_kernel.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_int, C.c_void_p,
                                    C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
    lib.ibf_batch_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p)]
    lib.ibf_apply_batch.argtypes = [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64), C.c_int, C.c_void_p]
    lib.ibf_batch_destroy.argtypes = [C.c_void_p]
    lib.ibf_build_batch.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_void_p,
                                    C.POINTER(C.c_int)]
    vp, i64, f32 = C.c_void_p, C.c_int64, C.c_float
    lib.ibf_dense_apply.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_int, vp, i64, vp, i64,
                                    vp, i64, vp, i64, i64, vp]
    lib.ibf_dense_apply_2d.argtypes = lib.ibf_dense_apply.argtypes
    lib.ibf_mlp_n_params.argtypes = [C.c_int]
    lib.ibf_mlp_features.argtypes = [i64, C.c_int, C.c_int, C.c_double, C.POINTER(C.c_float)]
    lib.ibf_mlp_forward.argtypes = [vp, C.c_int, vp, i64, vp, vp]
    lib.ibf_mlp_grad_work.argtypes = [C.c_int, i64]
    lib.ibf_mlp_grad_work.restype = i64
    lib.ibf_mlp_loss_grad.argtypes = [vp, C.c_int, vp, vp, i64, vp, vp, vp, vp]
    lib.ibf_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, f32, f32, f32, f32, vp]
    lib.ibf_mlp_select.argtypes = [vp, C.c_int, i64, C.c_int, C.c_double, C.c_double,
                                   C.c_int, C.c_int, C.POINTER(C.c_int),
                                   C.POINTER(C.c_double), vp]
    lib.ibf_tune.argtypes = [vp, vp, i64, vp, i64, i64, vp, C.POINTER(IBFTuning),
                             C.POINTER(IBFTuning)]
    lib.ibf_set_tuning.argtypes = [vp, i64, C.POINTER(IBFTuning)]
    lib.ibf_set_allocator.argtypes = [ALLOC_FN, FREE_FN]
    lib.ibf_measure_peak.argtypes = [C.c_int, vp, C.POINTER(C.c_double)]
    lib.ibf_apply_adjoint.argtypes = [vp, vp, i64, vp, i64, i64, vp]
    lib.ibf_apply_noalloc.argtypes = [vp, vp, i64, vp, i64, i64, vp]
    lib.ibf_rel_error.argtypes = [vp, i64, vp, i64, i64, i64, C.c_int, C.POINTER(C.c_double), vp]
    for name in ("ibf_plan", "ibf_build", "ibf_apply", "ibf_apply_profile", "ibf_query",
                 "ibf_destroy", "ibf_eval_kernel", "ibf_batch_create", "ibf_apply_batch",
                 "ibf_batch_destroy", "ibf_dense_apply", "ibf_mlp_n_params",
                 "ibf_mlp_features", "ibf_mlp_forward", "ibf_mlp_loss_grad", "ibf_mlp_adam",
                 "ibf_mlp_select", "ibf_tune", "ibf_set_tuning", "ibf_set_allocator", "ibf_measure_peak",
                 "ibf_apply_adjoint", "ibf_rel_error", "ibf_apply_noalloc",
                 "ibf_dense_apply_2d"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
# every allocator pair ever installed stays referenced: blocks it made are
# returned through it, possibly long after another pair was installed
_installed_allocators = []


def use_torch_allocator(enable: bool = True):
    """ibf_set_allocator with PyTorch's caching allocator (enable=True) or
    back to hipMalloc / hipFree (enable=False)."""
    lib = load()
    if not enable:
        _check(lib.ibf_set_allocator(ALLOC_FN(), FREE_FN()))
        return
    import torch

    def _alloc(nbytes, _stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device())
        except Exception:                      # reported as OOM by the library
            return None

    def _free(ptr, _stream):
        torch.cuda.caching_allocator_delete(ptr)

    pair = (ALLOC_FN(_alloc), FREE_FN(_free))
    _installed_allocators.append(pair)
    _check(lib.ibf_set_allocator(*pair))


PEAK_HBM_COPY, PEAK_MFMA_F32 = 0, 1


def build_batch(plans, nthreads: int = 0, stream=None):
    """ibf_build_batch: build the plans concurrently on worker streams.
    Returns the plans; raises IBFError naming the failed plan's index."""
    lib = load()
    arr = (C.c_void_p * len(plans))(*[pl.handle for pl in plans])
    failed = C.c_int(-1)
    rc = lib.ibf_build_batch(arr, len(plans), int(nthreads), _stream_handle(stream),
                             C.byref(failed))
    if rc != IBF_OK:
        raise IBFError(rc, f"plan {failed.value}: {last_error()}")
    return plans


def measure_peak(what: int, stream=None) -> float:
    """ibf_measure_peak: GB/s of a plain device copy (PEAK_HBM_COPY) or
    TFLOP/s of the FP32 4x4x1 MFMA loop (PEAK_MFMA_F32)."""
    lib = load()
    v = C.c_double()
    _check(lib.ibf_measure_peak(int(what), _stream_handle(stream), C.byref(v)))
    return float(v.value)


def last_error() -> str:
    return load().ibf_last_error().decode()


def _check(rc):
    if rc != IBF_OK:
        raise IBFError(rc, last_error())


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def make_desc(x, xi, phase, params, r, tol, leaf, precision, sweep_in=0,
              omega_lo=None, omega_width=0.0, device=0, fixed_ranks=None, amp=None,
              predictor=None, svd_sample=None):
    """Build an ibf_desc; returns (desc, keepalive) -- keep both alive.

    fixed_ranks: per-level rank caps (levels l0 .. L - l0) or None; amp:
    (amp_id, params) or None; predictor: (device float tensor, hidden width)
    for r <= 0, or None; svd_sample: (seed, samples) for the randomized
    low-rank approximation (dim 2), or None."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    prm = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    caps = None if fixed_ranks is None else np.ascontiguousarray(fixed_ranks, dtype=np.int32)
    aprm = np.ascontiguousarray(amp[1] if amp is not None else [], dtype=np.float64)
    d = IBFDesc()
    d.dim = 2 if x.ndim == 2 else 1
    d.n_x = x.shape[0]
    d.n_xi = xi.shape[0]
    d.x = x.ctypes.data_as(C.POINTER(C.c_double))
    d.xi = xi.ctypes.data_as(C.POINTER(C.c_double))
    if d.dim == 2:
        # Omega = [-W/2, W/2)^2; W defaults to the smallest power of two holding xi
        if not omega_width:
            m = float(np.max(np.abs(xi))) if xi.size else 1.0
            omega_width = 2.0 ** max(5, int(np.ceil(np.log2(2.0 * m + 1e-12))))
        omega_lo = -omega_width / 2.0
    d.omega_lo = float(-(xi.shape[0] // 2) if omega_lo is None else omega_lo)
    d.omega_width = float(omega_width)
    d.phase_id = int(phase)
    d.phase_params = prm.ctypes.data_as(C.POINTER(C.c_double)) if prm.size else None
    d.n_params = int(prm.size)
    d.r = int(r)
    d.tol = float(tol)
    d.leaf = int(leaf)
    d.precision = int(precision)
    d.sweep_in = int(sweep_in)
    d.device = int(device)
    d.fixed_ranks = caps.ctypes.data_as(C.POINTER(C.c_int)) if caps is not None else None
    d.amp_id = int(amp[0]) if amp is not None else 0
    d.amp_params = aprm.ctypes.data_as(C.POINTER(C.c_double)) if aprm.size else None
    d.n_amp_params = int(aprm.size)
    if predictor is not None:
        d.predictor = C.c_void_p(predictor[0].data_ptr())
        d.predictor_hidden = int(predictor[1])
    if svd_sample is not None:
        d.svd_seed = int(svd_sample[0]) & 0xFFFFFFFFFFFFFFFF
        d.svd_samples = int(svd_sample[1])
    return d, (x, xi, prm, caps, aprm)


class Plan:
    """Owns an ibf_plan_t.  Mirrors ibf_plan / ibf_build / ibf_apply /
    ibf_query / ibf_destroy; device vectors are torch tensors."""

    def __init__(self, x, xi, phase, params, r, tol, leaf=16, precision=PREC_FP64,
                 sweep_in=0, omega_lo=None, omega_width=0.0, device=0, fixed_ranks=None,
                 amp=None, predictor=None, svd_sample=None):
        lib = load()
        self._lib = lib
        d, keep = make_desc(x, xi, phase, params, r, tol, leaf, precision, sweep_in,
                            omega_lo, omega_width, device, fixed_ranks, amp, predictor,
                            svd_sample)
        # the predictor's parameters are read by ibf_build: keep them alive
        self._predictor = predictor
        h = C.c_void_p()
        _check(lib.ibf_plan(C.byref(d), C.byref(h)))
        self.handle = h
        self.precision = precision
        self.n_x = int(d.n_x)
        self.n_xi = int(d.n_xi)
        self.device = device

    @classmethod
    def from_problem(cls, P, precision=None, sweep_in=None, svd_sample=None):
        return cls(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf,
                   P.precision if precision is None else precision,
                   P.sweep_in if sweep_in is None else sweep_in,
                   omega_width=P.extra.get("omega_width", 0.0), svd_sample=svd_sample)

    def build(self, stream=None):
        _check(self._lib.ibf_build(self.handle, _stream_handle(stream)))
        return self

    def vector_dtype(self):
        import torch
        return torch.complex128 if self.precision == PREC_FP64 else torch.complex64

    def apply(self, g, u=None, stream=None):
        """g: device tensor (nrhs, n_xi) or (n_xi,), complex; returns u (nrhs, n_x)."""
        import torch
        squeeze = g.dim() == 1
        if squeeze:
            g = g.unsqueeze(0)
        if g.dtype != self.vector_dtype() or not g.is_contiguous():
            raise ValueError("g must be a contiguous tensor of the plan's complex dtype")
        nrhs = g.shape[0]
        if u is None:
            u = torch.empty((nrhs, self.n_x), dtype=g.dtype, device=g.device)
        _check(self._lib.ibf_apply(self.handle, C.c_void_p(g.data_ptr()), g.shape[1],
                                   C.c_void_p(u.data_ptr()), u.shape[1], nrhs,
                                   _stream_handle(stream)))
        return u[0] if squeeze else u

    def apply_adjoint(self, h, v=None, stream=None):
        """ibf_apply_adjoint: h device tensor (nrhs, n_x) or (n_x,); returns
        v = K^* h as (nrhs, n_xi)."""
        import torch
        squeeze = h.dim() == 1
        if squeeze:
            h = h.unsqueeze(0)
        if h.dtype != self.vector_dtype() or not h.is_contiguous():
            raise ValueError("h must be a contiguous tensor of the plan's complex dtype")
        nrhs = h.shape[0]
        if v is None:
            v = torch.empty((nrhs, self.n_xi), dtype=h.dtype, device=h.device)
        _check(self._lib.ibf_apply_adjoint(self.handle, C.c_void_p(h.data_ptr()), h.shape[1],
                                           C.c_void_p(v.data_ptr()), v.shape[1], nrhs,
                                           _stream_handle(stream)))
        return v[0] if squeeze else v

    def apply_noalloc(self, g, u, stream=None):
        """ibf_apply_noalloc on (nrhs, n) tensors (u preallocated): the same
        product with the coefficient buffers in the library's static scratch
        array (no device allocation)."""
        if g.dtype != self.vector_dtype() or not g.is_contiguous() or not u.is_contiguous():
            raise ValueError("g and u must be contiguous tensors of the plan's complex dtype")
        _check(self._lib.ibf_apply_noalloc(self.handle, C.c_void_p(g.data_ptr()), g.shape[1],
                                           C.c_void_p(u.data_ptr()), u.shape[1], g.shape[0],
                                           _stream_handle(stream)))
        return u

    def apply_raw(self, g_ptr, ldg, u_ptr, ldu, nrhs, stream=None):
        _check(self._lib.ibf_apply(self.handle, C.c_void_p(g_ptr), ldg, C.c_void_p(u_ptr), ldu,
                                   nrhs, _stream_handle(stream)))

    def tune(self, g, u=None, stream=None) -> dict:
        """ibf_tune on (nrhs, n) tensors: times the candidate schedules, keeps
        the fastest for later applies with this nrhs (u receives the product);
        returns the choice and the default rule's time."""
        import torch
        if g.dtype != self.vector_dtype() or not g.is_contiguous() or g.dim() != 2:
            raise ValueError("g must be a contiguous (nrhs, n) tensor of the plan's complex dtype")
        if u is None:
            u = torch.empty((g.shape[0], self.n_x), dtype=g.dtype, device=g.device)
        best, dflt = IBFTuning(), IBFTuning()
        _check(self._lib.ibf_tune(self.handle, C.c_void_p(g.data_ptr()), g.shape[1],
                                  C.c_void_p(u.data_ptr()), u.shape[1], g.shape[0],
                                  _stream_handle(stream), C.byref(best), C.byref(dflt)))
        return {"path": PATHS[best.path], "chunk": best.chunk,
                "max_fused": best.max_fused, "split": best.split, "ms": float(best.ms),
                "default_ms": float(dflt.ms)}

    def set_tuning(self, nrhs, path=None, chunk=0, max_fused=0, split=0):
        """ibf_set_tuning: installs a schedule for `nrhs` right-hand sides
        (path "default", "vector", "mfma", "tight" -- MFMA stages at each
        pair's own ranks -- or "tight_split" -- the same with BF16 split
        products, BF16X2 plans); path None returns to the default rule."""
        if path is None:
            _check(self._lib.ibf_set_tuning(self.handle, nrhs, None))
            return
        t = IBFTuning(PATHS.index(path), chunk, max_fused, 0.0, split)
        _check(self._lib.ibf_set_tuning(self.handle, nrhs, C.byref(t)))

    def apply_profile(self, g, u, stream=None):
        """ibf_apply_profile on (nrhs, n) tensors; returns a list of launches
        (name, ms, flops, bytes, vec_bytes)."""
        prof = IBFProfile()
        _check(self._lib.ibf_apply_profile(self.handle, C.c_void_p(g.data_ptr()), g.shape[1],
                                           C.c_void_p(u.data_ptr()), u.shape[1], g.shape[0],
                                           _stream_handle(stream), C.byref(prof)))
        return [(bytes(prof.name[i]).split(b"\0")[0].decode(), float(prof.ms[i]),
                 float(prof.flops[i]), float(prof.bytes[i]), float(prof.vec_bytes[i]))
                for i in range(prof.n_launches)]

    def query(self) -> dict:
        info = IBFInfo()
        _check(self._lib.ibf_query(self.handle, C.byref(info)))
        n = info.n_levels
        return {
            "L": info.L, "l0": info.l0, "h": info.h, "n_levels": n,
            "rank": [info.rank[i] for i in range(n)],
            "n_pairs": info.n_pairs, "nnz_prelim": info.nnz_prelim,
            "nnz_opt": info.nnz_opt, "nnz_stored": info.nnz_stored,
            "factor_bytes": info.factor_bytes, "build_ms": info.build_ms,
            "smax_x": info.smax_x, "smax_xi": info.smax_xi,
            "R_comp": info.nnz_prelim / max(info.nnz_opt, 1),
            "sweep_in": info.sweep_in,
            "rank_in_g": [info.rank_in_g[i] for i in range(n)],
            "rank_in_h": [info.rank_in_h[i] for i in range(n)],
            "r": info.r, "tol": info.tol, "learned": info.learned,
        }

    def destroy(self):
        if getattr(self, "handle", None):
            self._lib.ibf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """ibf_batch_create / ibf_apply_batch over built plans (kept alive here)."""

    def __init__(self, plans):
        self._lib = load()
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[p.handle for p in self.plans])
        h = C.c_void_p()
        _check(self._lib.ibf_batch_create(arr, len(self.plans), C.byref(h)))
        self.handle = h

    def apply(self, gs, us=None, graph=True, stream=None):
        """gs: list of device tensors (nrhs_i, n_xi_i); returns the list of u_i (nrhs_i, n_x_i)."""
        import torch
        n = len(self.plans)
        if len(gs) != n:
            raise ValueError("one g per plan")
        if us is None:
            us = [torch.empty((g.shape[0], p.n_x), dtype=g.dtype, device=g.device)
                  for g, p in zip(gs, self.plans)]
        for g, u, p in zip(gs, us, self.plans):
            if g.dtype != p.vector_dtype() or not g.is_contiguous() or not u.is_contiguous():
                raise ValueError("g and u must be contiguous tensors of the plans' complex dtype")
        gp = (C.c_void_p * n)(*[g.data_ptr() for g in gs])
        up = (C.c_void_p * n)(*[u.data_ptr() for u in us])
        ldg = (C.c_int64 * n)(*[g.shape[1] for g in gs])
        ldu = (C.c_int64 * n)(*[u.shape[1] for u in us])
        nr = (C.c_int64 * n)(*[g.shape[0] for g in gs])
        _check(self._lib.ibf_apply_batch(self.handle, gp, ldg, up, ldu, nr,
                                         BATCH_GRAPH if graph else 0, _stream_handle(stream)))
        return us

    def destroy(self):
        if getattr(self, "handle", None):
            self._lib.ibf_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def eval_kernel(phase, params, x_dev, xi_dev, stream=None):
    """exp(2 pi i Phi(x, xi)) on the device for paired float64 tensors."""
    import torch
    lib = load()
    prm = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    out = torch.empty(x_dev.shape[0], dtype=torch.complex128, device=x_dev.device)
    _check(lib.ibf_eval_kernel(int(phase),
                               prm.ctypes.data_as(C.POINTER(C.c_double)) if prm.size else None,
                               int(prm.size), C.c_void_p(x_dev.data_ptr()),
                               C.c_void_p(xi_dev.data_ptr()), x_dev.shape[0],
                               C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


def dense_apply(phase, params, x_dev, xi_dev, g, stream=None):
    """Device FP64 direct product: g (nrhs, n_xi) complex128 -> u (nrhs, n_x)."""
    import torch
    lib = load()
    prm = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    nrhs = g.shape[0]
    u = torch.empty((nrhs, x_dev.shape[0]), dtype=torch.complex128, device=g.device)
    _check(lib.ibf_dense_apply(int(phase),
                               prm.ctypes.data_as(C.POINTER(C.c_double)) if prm.size else None,
                               int(prm.size), C.c_void_p(x_dev.data_ptr()), x_dev.shape[0],
                               C.c_void_p(xi_dev.data_ptr()), xi_dev.shape[0],
                               C.c_void_p(g.data_ptr()), g.shape[1], C.c_void_p(u.data_ptr()),
                               u.shape[1], nrhs, _stream_handle(stream)))
    return u


def dense_apply_2d(phase, params, x_dev, xi_dev, g, stream=None):
    """Device FP64 direct 2-D product: x (n_x, 2), xi (n_xi, 2) float64 device
    tensors, g (nrhs, n_xi) complex128 -> u (nrhs, n_x)."""
    import torch
    lib = load()
    prm = np.ascontiguousarray(params if params is not None else [], dtype=np.float64)
    nrhs = g.shape[0]
    u = torch.empty((nrhs, x_dev.shape[0]), dtype=torch.complex128, device=g.device)
    _check(lib.ibf_dense_apply_2d(int(phase),
                                  prm.ctypes.data_as(C.POINTER(C.c_double)) if prm.size else None,
                                  int(prm.size), C.c_void_p(x_dev.data_ptr()), x_dev.shape[0],
                                  C.c_void_p(xi_dev.data_ptr()), xi_dev.shape[0],
                                  C.c_void_p(g.data_ptr()), g.shape[1], C.c_void_p(u.data_ptr()),
                                  u.shape[1], nrhs, _stream_handle(stream)))
    return u


def rel_error(u, ref, stream=None):
    """ibf_rel_error on (nrhs, n) device tensors of one complex dtype:
    (Frobenius relative error over all columns, largest per-column one)."""
    if u.shape != ref.shape or u.dtype != ref.dtype:
        raise ValueError("u and ref must have the same shape and dtype")
    if u.dim() == 1:
        u, ref = u.unsqueeze(0), ref.unsqueeze(0)
    import torch
    prec = PREC_FP64 if u.dtype == torch.complex128 else PREC_FP32
    u, ref = u.contiguous(), ref.contiguous()
    out = (C.c_double * 2)()
    _check(load().ibf_rel_error(C.c_void_p(u.data_ptr()), u.shape[1], C.c_void_p(ref.data_ptr()),
                                ref.shape[1], u.shape[1], u.shape[0], prec, out,
                                _stream_handle(stream)))
    return float(out[0]), float(out[1])


def mlp_n_params(n_hidden):
    n = load().ibf_mlp_n_params(n_hidden)
    if n < 0:
        raise ValueError(f"unsupported hidden width {n_hidden}")
    return n


def mlp_features(n, phase, r, tol):
    out = (C.c_float * MLP_FEATURES)()
    _check(load().ibf_mlp_features(int(n), int(phase), int(r), float(tol), out))
    return np.array(out[:], dtype=np.float32)


def mlp_forward(params, n_hidden, X, stream=None):
    import torch
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(load().ibf_mlp_forward(C.c_void_p(params.data_ptr()), n_hidden,
                                  C.c_void_p(X.data_ptr()), X.shape[0], C.c_void_p(y.data_ptr()),
                                  _stream_handle(stream)))
    return y


def mlp_loss_grad(params, n_hidden, X, T, stream=None):
    """(loss, grad) device tensors for the mean squared error over the samples."""
    import torch
    lib = load()
    n = X.shape[0]
    work = torch.empty(lib.ibf_mlp_grad_work(n_hidden, n), dtype=torch.float32, device=X.device)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib.ibf_mlp_loss_grad(C.c_void_p(params.data_ptr()), n_hidden,
                                 C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
                                 C.c_void_p(grad.data_ptr()), C.c_void_p(loss.data_ptr()),
                                 C.c_void_p(work.data_ptr()), _stream_handle(stream)))
    return loss, grad


def mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().ibf_mlp_adam(C.c_void_p(params.data_ptr()), C.c_void_p(grad.data_ptr()),
                               C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()),
                               params.numel(), int(step), lr, beta1, beta2, eps,
                               _stream_handle(stream)))


def mlp_select(params, n_hidden, n, phase, tol, margin=0.3, rmin=2, rmax=16, stream=None):
    """(r, svd_tol) predicted to meet tol, or (0, tol) when none qualifies."""
    r = C.c_int(0)
    st = C.c_double(0.0)
    _check(load().ibf_mlp_select(C.c_void_p(params.data_ptr()), n_hidden, int(n), int(phase),
                                 float(tol), float(margin), rmin, rmax, C.byref(r), C.byref(st),
                                 _stream_handle(stream)))
    return r.value, st.value
