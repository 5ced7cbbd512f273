"""IBF apply throughput on one MI355X.

Default workload: the 1-D FIO of the paper's Sec. 6.2 at N = 65536 (uniform
grids, c(x) = (2 + sin 2 pi x)/8), r = 12, tol = 1e-6, leaf 16, 64 complex
normal right-hand sides from seed 1, complex FP32 factors and apply.
A step is one application of the compressed IBF to the 64-column batch,
inputs already resident in HBM.  Reported alongside: build ms, the relative
error against the plain FP64 IBF (same factorization settings) and against
the dense product on 256 sampled rows, the plain FP64 single-RHS apply rate,
the roofline of the dominant kernel and the CPU oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload fio1d_64k|nudft_1m|fio1d_1k] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFS = 157.3          # MI355X dense FP32 (matrix)
FP64_PEAK_TFS = 78.6
BF16_PEAK_TFS = 2500.0


def _workload(name, nrhs=None):
    from paper_1605_03616_amd import inputs as I
    if name == "fio1d_64k":
        return I.workload_fio1d_64k(nrhs=nrhs or 64)
    if name == "nudft_1m":
        return I.workload_nudft_1m(nrhs=nrhs or 16)
    if name == "fio1d_1k":
        return I.workload_fio1d_1k()
    raise SystemExit(f"unknown workload {name}")


def _roofline(launches, bound, peak, unit):
    """Aggregate the dominant kernel class over profiled launches."""
    by = {}
    for name, ms, flops, byts in launches:
        d = by.setdefault(name, [0.0, 0.0, 0.0, 0])
        d[0] += ms
        d[1] += flops
        d[2] += byts
        d[3] += 1
    dom = max(by, key=lambda k: by[k][0])
    ms, flops, byts, cnt = by[dom]
    if bound == "mfma":
        achieved = flops / (ms * 1e-3) / 1e12
    else:
        achieved = byts / (ms * 1e-3) / 1e9
    return dom, {
        "kernel": dom,
        "bound": bound,
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": None,
        "launches": cnt,
        "avg_launch_ms": round(ms / cnt, 5),
        "algorithmic_flops_per_launch": flops / cnt,
        "algorithmic_bytes_per_launch": byts / cnt,
    }, {k: {"ms": round(v[0], 4), "launches": v[3]} for k, v in by.items()}


def _cpu_baseline(P, nrhs_sample=4):
    """Time the FP64 oracle's IBF apply on the host: full oracle build (not
    timed), then the apply of `nrhs_sample` columns, scaled to the metric."""
    from oracle import ibf_oracle as O
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([d.get("num_threads", 1) for d in info] or [1])
    except Exception:
        cores = os.cpu_count()
    t0 = time.perf_counter()
    prob, F, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf)
    t_build = time.perf_counter() - t0
    g = P.g[:, :nrhs_sample]
    t0 = time.perf_counter()
    O.apply_optimal(Op, g)
    t_app = time.perf_counter() - t0
    return {
        "value": round(P.n * nrhs_sample / t_app / 1e9, 8),
        "unit": "G(complex samples*RHS)/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"numpy FP64 oracle IBF apply of {nrhs_sample} of the {P.nrhs} RHS at "
                  f"N={P.n}, r={P.r} (oracle build {t_build:.1f} s not included)",
        "apply_s": round(t_app, 3),
        "build_s": round(t_build, 2),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fio1d_64k")
    ap.add_argument("--nrhs", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 256 MiB elementwise copy first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "the IBF path here is single-GPU", file=sys.stderr)
        sys.exit(2)

    import torch

    from oracle import ibf_oracle as O
    from paper_1605_03616_amd import ibf
    from paper_1605_03616_amd import inputs as I

    ibf.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    P = _workload(args.workload, args.nrhs)
    dt = torch.complex128 if P.precision == I.PREC_FP64 else torch.complex64
    print(f"[bench] workload {P.name} N={P.n} r={P.r} nrhs={P.nrhs} precision={P.precision}",
          file=sys.stderr, flush=True)

    pl = ibf.Plan.from_problem(P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl.build()
    build_wall_ms = (time.perf_counter() - t0) * 1e3
    q = pl.query()
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(dt).cuda()
    u = torch.empty((P.nrhs, P.n), dtype=dt, device="cuda")
    stream = torch.cuda.current_stream()

    if args.calib_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)          # reads 256 MiB, writes 256 MiB
        torch.cuda.synchronize()
        del a, b
    for _ in range(args.warmup):
        pl.apply(g, u)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        pl.apply(g, u)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = P.n * P.nrhs / (ms * 1e-3) / 1e9
    print(f"[bench] timed {args.steps} steps: {ms:.4f} ms/step", file=sys.stderr, flush=True)

    # per-kernel HIP-event timings over a second timed region on the same stream
    launches = []
    for _ in range(max(3, args.steps // 4)):
        launches += pl.apply_profile(g, u)
    if P.precision == I.PREC_FP64:
        bound, peak = ("hbm", HBM_PEAK_GBS) if P.nrhs < 8 else ("mfma", FP64_PEAK_TFS)
    elif P.precision == I.PREC_FP32:
        bound, peak = ("mfma", FP32_PEAK_TFS) if P.nrhs >= 32 else ("hbm", HBM_PEAK_GBS)
    else:
        bound, peak = ("hbm", HBM_PEAK_GBS) if P.nrhs < 64 else ("mfma", BF16_PEAK_TFS)
    unit = "TFLOP/s" if bound == "mfma" else "GB/s"
    dom, roof, per_class = _roofline(launches, bound, peak, unit)

    out = {
        "metric": "IBF apply G(complex samples*RHS)/s at rel err 1e-5 vs plain FP64; build ms",
        "value": round(value, 4),
        "unit": "G(complex samples*RHS)/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {I.PREC_FP64: "f64", I.PREC_FP32: "f32", I.PREC_BF16X2: "bf16x2+f32"}[P.precision],
        "data": "synthetic",
        "config": {"workload": P.name, "N": P.n, "r": P.r, "nrhs": P.nrhs, "tol": P.tol,
                   "leaf": P.leaf, "phase": P.phase, "parallelism": "single-gpu"},
        "build_ms": round(q["build_ms"], 3),
        "build_wall_ms": round(build_wall_ms, 3),
        "ranks": q["rank"],
        "R_comp": round(q["R_comp"], 4),
        "nnz_opt": q["nnz_opt"],
        "nnz_stored": q["nnz_stored"],
        "factor_bytes": q["factor_bytes"],
        "kernel_ms_per_step": {k: round(v["ms"] / max(3, args.steps // 4), 4)
                               for k, v in per_class.items()},
        "roofline": roof,
    }

    if not args.no_accuracy:
        # plain FP64 IBF on the same input: accuracy reference and single-RHS rate
        pl64 = ibf.Plan.from_problem(P, precision=I.PREC_FP64)
        pl64.build()
        g64 = torch.from_numpy(np.ascontiguousarray(P.g.T)).cuda()
        u64 = pl64.apply(g64)
        torch.cuda.synchronize()
        uu = u.to(torch.complex128)
        out["rel_err_vs_fp64"] = float(torch.linalg.norm(uu - u64) / torch.linalg.norm(u64))
        g1 = g64[:1].contiguous()
        u1 = torch.empty((1, P.n), dtype=torch.complex128, device="cuda")
        for _ in range(3):
            pl64.apply(g1, u1)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            pl64.apply(g1, u1)
        e1.record(stream)
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1) / args.steps
        out["fp64_single_rhs"] = {"ms": round(ms1, 5), "value": round(P.n / (ms1 * 1e-3) / 1e9, 5),
                                  "build_ms": round(pl64.query()["build_ms"], 3)}
        pl64.destroy()
        rows = I.error_rows(P.n)
        nchk = min(P.nrhs, 4)
        ud = O.dense_apply(P.phase, P.params, P.x, P.xi, P.g[:, :nchk], rows=rows)
        un = u[:nchk].cpu().numpy().T[rows]
        out["rel_err_vs_dense_sampled"] = O.rel_error(un, ud)

    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(P)
    pl.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
