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
                       [--workload fio1d_64k|nudft_1m|fio1d_1k|batched|fio2d_256] [--no-cpu-baseline]
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


# HBM traffic of the dominant apply kernel measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch), each scaled by what the
# counter reads for a plain 256 MiB elementwise copy (FETCH_SIZE reads half
# the bytes read: x2.0; WRITE_SIZE reads the bytes written: x1.0).  Valid only
# for the apply source it was measured on: any change to it voids the figure.
APPLY_SRC = os.path.join(ROOT, "paper_1605_03616_amd", "csrc", "ibf_apply.hip")
MEASURED_TRAFFIC = {
    # (workload, schedule path/chunk/max_fused) -> (sha1 of the apply source,
    #   kernel class, [(launches per step, FETCH_SIZE KiB, WRITE_SIZE KiB), ...])
    ("fio1d_n65536_r12_fp32", "default/0/0"): (
        "dd691557a76f9a3356f790409089cd4c61c16094", "apply_stage_tight",
        [(2, 323079, 238008)]),
    ("fio1d_n65536_r12_bf16x2", "default/0/0"): (
        "dd691557a76f9a3356f790409089cd4c61c16094", "apply_stage_tight_split",
        [(2, 311345, 236984)]),
    ("nudft_n1048576_r10", "default/0/0"): (
        "dd691557a76f9a3356f790409089cd4c61c16094", "apply_fused_mfma",
        [(2, 2424919, 983040), (1, 1769577, 917504), (1, 1822846, 1048576)]),
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def _measured_traffic(workload, schedule, kernel):
    """Average HBM bytes per launch of `kernel`, or None if not measured for
    this exact apply source and schedule."""
    import hashlib
    ent = MEASURED_TRAFFIC.get((workload, schedule))
    if not ent or ent[1] != kernel:
        return None
    with open(APPLY_SRC, "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != ent[0]:
            return None
    n = sum(c for c, _, _ in ent[2])
    tot = sum(c * (fk * FETCH_SCALE + wk * WRITE_SCALE) * 1024.0 for c, fk, wk in ent[2])
    return tot / n


def _workload(name, nrhs=None, precision=None):
    """The named workload; `precision` ("fp32", "bf16x2", "fp64") replaces
    the storage precision of its factors (the workload name then carries it)."""
    import dataclasses

    from paper_1605_03616_amd import inputs as I
    if name == "fio1d_64k":
        P = I.workload_fio1d_64k(nrhs=nrhs or 64)
    elif name == "nudft_1m":
        P = I.workload_nudft_1m(nrhs=nrhs or 16)
    elif name == "fio1d_1k":
        P = I.workload_fio1d_1k()
    else:
        raise SystemExit(f"unknown workload {name}")
    if precision:
        prec = {"fp64": I.PREC_FP64, "fp32": I.PREC_FP32, "bf16x2": I.PREC_BF16X2}[precision]
        if prec != P.precision:
            base = P.name[:-5] if P.name.endswith("_fp32") else P.name
            P = dataclasses.replace(P, precision=prec, name=f"{base}_{precision}")
    return P


def _roofline(launches, bound, peak, unit):
    """Aggregate the dominant kernel class over profiled launches."""
    by = {}
    for name, ms, flops, byts, vbytes in launches:
        d = by.setdefault(name, [0.0, 0.0, 0.0, 0, 0.0])
        d[0] += ms
        d[1] += flops
        d[2] += byts
        d[3] += 1
        d[4] += vbytes
    dom = max(by, key=lambda k: by[k][0])
    ms, flops, byts, cnt, vbytes = by[dom]
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
        # factors (unpadded) plus the samples g / u the launch reads or writes
        "algorithmic_bytes_per_launch": byts / cnt,
        # intermediate coefficient vectors at their stored ranks: the design's
        # launch-boundary traffic, not algorithmic
        "vector_bytes_per_launch": vbytes / cnt,
    }, {k: {"ms": round(v[0], 4), "launches": v[3]} for k, v in by.items()}


def _cpu_baseline(P, nrhs_sample=20):
    """Time the FP64 oracle's IBF apply on the host: full oracle build (not
    timed), then the apply of `nrhs_sample` columns, scaled to the metric."""
    from oracle import ibf_oracle as O
    cores = _cores()
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


def _bench_batched(args):
    """Uneven batch of 256 1-D FIO problems, one graph-replayed batched apply per step."""
    import torch
    from paper_1605_03616_amd import ibf
    from paper_1605_03616_amd import inputs as I

    ibf.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    learned = args.batch_r == "mlp"
    probs = I.workload_batched(count=args.batch_count, seed=3,
                               r=12 if learned else int(args.batch_r))
    print(f"[bench] batched workload: {len(probs)} problems, sum N = {sum(P.n for P in probs)}",
          file=sys.stderr, flush=True)
    pred_info = None
    if learned:
        # orders (and truncation) from the learned predictor for the 1e-6 target,
        # trained here on the device from the factorization's own error data
        from paper_1605_03616_amd import predictor as PR
        t0 = time.perf_counter()
        data = PR.generate(PR.default_sizes())
        t_data = time.perf_counter() - t0
        pred = PR.Predictor(n_hidden=16, seed=5)
        t0 = time.perf_counter()
        loss = pred.fit(data)
        t_fit = time.perf_counter() - t0
        choice = [pred.select(P.n, P.phase, 1e-6) for P in probs]
        for P, (r, st) in zip(probs, choice):
            P.r, P.tol = r, st
        rs = [c[0] for c in choice]
        pred_info = {"samples": len(data.Y), "data_s": round(t_data, 2),
                     "train_s": round(t_fit, 2), "train_loss": loss,
                     "r_hist": {int(r): rs.count(r) for r in sorted(set(rs))},
                     "truncations": sorted({f"{c[1]:.2g}" for c in choice})}
        print(f"[bench] predictor: {pred_info}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the plans are independent: built concurrently, one HIP stream per host thread
    plans = ibf.build_batch([ibf.Plan.from_problem(P) for P in probs])
    build_s = time.perf_counter() - t0
    qs = [pl.query() for pl in plans]
    gs = [torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda() for P in probs]
    us = [torch.empty((P.nrhs, P.n), dtype=torch.complex64, device="cuda") for P in probs]
    tune_info = None
    if args.schedule:        # one installed schedule for every plan
        f = args.schedule.split("/")
        for pl, P in zip(plans, probs):
            pl.set_tuning(P.nrhs, f[0], int(f[1]), int(f[2]), int(f[3]) if len(f) > 3 else 0)
        tune_info = {"fixed": args.schedule}
    elif not args.no_tune:   # schedule autotuner per plan, before the timed region
        t0 = time.perf_counter()
        picks = [pl.tune(g, u) for pl, g, u in zip(plans, gs, us)]
        torch.cuda.synchronize()
        kinds = [f"{t['path']}/{t['chunk']}/{t['max_fused']}" + (f"/{t['split']}" if t['split'] else "") for t in picks]
        tune_info = {"tune_s": round(time.perf_counter() - t0, 3),
                     "choices": {k: kinds.count(k) for k in sorted(set(kinds))}}
        print(f"[bench] tuning: {tune_info}", file=sys.stderr, flush=True)
    B = ibf.Batch(plans)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        B.apply(gs, us, graph=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        B.apply(gs, us, graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    units = sum(P.n * P.nrhs for P in probs)
    value = units / (ms * 1e-3) / 1e9
    # algorithmic bytes: unpadded FP32 factors once + input and output samples
    abytes = sum(8.0 * q["nnz_opt"] + 16.0 * P.n * P.nrhs for q, P in zip(qs, probs))
    achieved = abytes / (ms * 1e-3) / 1e9
    out = {
        "metric": "IBF apply G(complex samples*RHS)/s at rel err 1e-5 vs plain FP64; build ms",
        "value": round(value, 4),
        "unit": "G(complex samples*RHS)/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched_fio1d_{len(probs)}_problems_r{args.batch_r}",
                   "target_tol": 1e-6,
                   "count": len(probs), "sum_N": sum(P.n for P in probs),
                   "sum_N_x_nrhs": units, "parallelism": "single-gpu"},
        "build_ms": round(build_s * 1e3, 3),
        "build_ms_sum_over_plans": round(sum(q["build_ms"] for q in qs), 3),
        "nnz_opt": sum(q["nnz_opt"] for q in qs),
        "roofline": {"kernel": "whole batched apply (graph of phase launches)", "bound": "hbm",
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_step": abytes},
    }
    if pred_info:
        out["predictor"] = pred_info
    if tune_info:
        out["tuning"] = tune_info
    if not args.no_accuracy:
        # the library's device FP64 direct product on 64 sampled rows a problem
        worst = 0.0
        for P, u in zip(probs, us):
            rows = I.error_rows(P.n, count=64)
            ud = ibf.dense_apply(P.phase, P.params,
                                 torch.from_numpy(np.ascontiguousarray(P.x[rows])).cuda(),
                                 torch.from_numpy(np.ascontiguousarray(P.xi)).cuda(),
                                 torch.from_numpy(np.ascontiguousarray(P.g.T)).cuda())
            un = u[:, torch.from_numpy(rows).cuda()].to(torch.complex128).contiguous()
            worst = max(worst, ibf.rel_error(un, ud)[0])
        out["max_rel_err_vs_dense_sampled"] = worst
    if not args.no_cpu_baseline:
        from oracle import ibf_oracle as O
        small = [P for P in probs if P.n <= 2048][:8]
        t_app = 0.0
        for P in small:
            _, _, Op = O.build_optimal(P.phase, P.params, P.x, P.xi, P.r, P.tol, P.leaf,
                                       sweep_in_on=False)
            t0 = time.perf_counter()
            O.apply_optimal(Op, P.g)
            t_app += time.perf_counter() - t0
        su = sum(P.n * P.nrhs for P in small)
        out["cpu_baseline"] = {"value": round(su / t_app / 1e9, 8),
                               "unit": "G(complex samples*RHS)/s", "cores": _cores(),
                               "kind": "oracle",
                               "sample": f"numpy FP64 oracle IBF apply of the {len(small)} "
                                         f"problems of the batch with N <= 2048 (build not timed)"}
    B.destroy()
    for pl in plans:
        pl.destroy()
    print(json.dumps(out), flush=True)


def _bench_2d(args):
    """2-D FIO on the 256 x 256 grid (multiscale IBF, r = 5 x 5, tol 1e-4, 8 RHS, FP32)."""
    import torch
    from paper_1605_03616_amd import ibf
    from paper_1605_03616_amd import inputs as I

    ibf.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    P = I.workload_fio2d_256(nrhs=args.nrhs or 8)
    print(f"[bench] workload {P.name} N={P.n} r={P.r} nrhs={P.nrhs}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pl = ibf.Plan.from_problem(P).build()
    build_wall = (time.perf_counter() - t0) * 1e3
    q = pl.query()
    g = torch.from_numpy(np.ascontiguousarray(P.g.T)).to(torch.complex64).cuda()
    u = torch.empty((P.nrhs, P.n), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream()
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
    abytes = 8.0 * q["nnz_opt"] + 16.0 * P.n * P.nrhs
    achieved = abytes / (ms * 1e-3) / 1e9
    out = {
        "metric": "IBF apply G(complex samples*RHS)/s at rel err 1e-5 vs plain FP64; build ms",
        "value": round(P.n * P.nrhs / (ms * 1e-3) / 1e9, 4),
        "unit": "G(complex samples*RHS)/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": P.name, "N": P.n, "grid": "256x256", "r": "5x5", "nrhs": P.nrhs,
                   "tol": P.tol, "phase": P.phase, "parallelism": "single-gpu"},
        "build_ms": round(q["build_ms"], 3), "build_wall_ms": round(build_wall, 3),
        "nnz_prelim": q["nnz_prelim"], "nnz_opt": q["nnz_opt"], "R_comp": round(q["R_comp"], 4),
        "factor_bytes": q["factor_bytes"],
        "roofline": {"kernel": "whole multiscale apply (centre + 48 box IBFs)", "bound": "hbm",
                     "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_step": abytes},
    }
    if not args.no_accuracy:
        pl64 = ibf.Plan.from_problem(P, precision=I.PREC_FP64).build()
        u64 = pl64.apply(torch.from_numpy(np.ascontiguousarray(P.g.T)).cuda())
        out["rel_err_vs_fp64"] = ibf.rel_error(u.to(torch.complex128), u64)[0]
        out["fp64_build_ms"] = round(pl64.query()["build_ms"], 3)
        pl64.destroy()
        # the library's device FP64 direct 2-D product on 256 sampled rows
        rows = np.random.default_rng(1234).choice(P.n, 256, replace=False)
        ud = ibf.dense_apply_2d(P.phase, P.params,
                                torch.from_numpy(np.ascontiguousarray(P.x[rows])).cuda(),
                                torch.from_numpy(np.ascontiguousarray(P.xi)).cuda(),
                                torch.from_numpy(np.ascontiguousarray(P.g[:, :2].T)).cuda())
        un = u[:2][:, torch.from_numpy(rows).cuda()].to(torch.complex128).contiguous()
        out["rel_err_vs_dense_sampled"] = ibf.rel_error(un, ud)[0]
    if not args.no_cpu_baseline:
        # the oracle MIBF apply on the 64 x 64 grid of the same workload (build not timed)
        from oracle import ibf2d_oracle as D
        Ps = I.fio2d_grid(64, 5, P.nrhs, 3, tol=1e-4)
        part, built, cidx = D.mibf_build(Ps.phase, Ps.params, Ps.x, Ps.xi, 64, 5, 1e-4)
        t0 = time.perf_counter()
        D.mibf_apply(Ps.phase, Ps.params, Ps.x, Ps.xi, Ps.g, built, cidx)
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(Ps.n * Ps.nrhs / t / 1e9, 8),
                               "unit": "G(complex samples*RHS)/s", "cores": _cores(),
                               "kind": "oracle",
                               "sample": "numpy FP64 oracle MIBF apply on the 64 x 64 grid of the "
                                         "same 2-D FIO (r = 5, tol 1e-4, 8 RHS), build not timed"}
    pl.destroy()
    print(json.dumps(out), flush=True)


def _cores():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return max([d.get("num_threads", 1) for d in info] or [1])
    except Exception:
        return os.cpu_count()


def _bench_adjoint(args):
    """The adjoint apply v = K^* h on a 1-D workload (built as the forward
    bench builds it, the sweep-in included): throughput, the whole-step
    roofline, and the error against the FP64 adjoint of the same
    factorization."""
    import torch

    from paper_1605_03616_amd import ibf
    from paper_1605_03616_amd import inputs as I

    ibf.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    P = _workload(args.workload, args.nrhs, args.precision)
    dt = torch.complex128 if P.precision == I.PREC_FP64 else torch.complex64
    sw = int(getattr(P, "sweep_in", 0) or 0)
    pl = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, P.precision, sw).build()
    q = pl.query()
    rng = np.random.default_rng(7)
    h = I.complex_normal(P.n, P.nrhs, rng)
    ht = torch.from_numpy(np.ascontiguousarray(h.T)).to(dt).cuda()
    v = torch.empty((P.nrhs, P.n), dtype=dt, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        pl.apply_adjoint(ht, v)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        pl.apply_adjoint(ht, v)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    flops = 8.0 * q["nnz_opt"] * P.nrhs
    bound, peak, unit = (("mfma", FP32_PEAK_TFS, "TFLOP/s") if P.nrhs >= 32 else
                         ("hbm", HBM_PEAK_GBS, "GB/s"))
    fb = 16.0 if P.precision == I.PREC_FP64 else 8.0
    byts = fb * q["nnz_opt"] + 2 * fb * P.n * P.nrhs
    achieved = flops / (ms * 1e-3) / 1e12 if bound == "mfma" else byts / (ms * 1e-3) / 1e9
    out = {
        "metric": "IBF adjoint apply G(complex samples*RHS)/s (v = K^* h)",
        "value": round(P.n * P.nrhs / (ms * 1e-3) / 1e9, 4),
        "unit": "G(complex samples*RHS)/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {I.PREC_FP64: "f64", I.PREC_FP32: "f32", I.PREC_BF16X2: "bf16x2+f32"}[P.precision],
        "data": "synthetic",
        "config": {"workload": P.name + "_adjoint", "N": P.n, "r": P.r, "nrhs": P.nrhs,
                   "tol": P.tol, "sweep_in": q["sweep_in"], "parallelism": "single-gpu"},
        "roofline": {"kernel": "whole adjoint apply", "bound": bound,
                     "achieved": round(achieved, 3), "peak": peak, "unit": unit,
                     "frac": round(achieved / peak, 4), "traffic": None},
    }
    if not args.no_accuracy and P.precision != I.PREC_FP64:
        pl64 = ibf.Plan(P.x, P.xi, P.phase, P.params, P.r, P.tol, P.leaf, I.PREC_FP64, sw).build()
        v64 = pl64.apply_adjoint(torch.from_numpy(np.ascontiguousarray(h.T)).cuda())
        torch.cuda.synchronize()
        a = v.cpu().numpy().astype(np.complex128)
        b = v64.cpu().numpy()
        out["rel_err_vs_fp64"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        pl64.destroy()
    pl.destroy()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps first (the clocks ramp up over the first ~0.1 s)")
    ap.add_argument("--workload", default="fio1d_64k")
    ap.add_argument("--nrhs", type=int, default=None)
    ap.add_argument("--precision", choices=["fp32", "bf16x2", "fp64"], default=None,
                    help="factor storage precision in place of the workload's own (1-D)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the schedule autotuner (apply with the default rule)")
    ap.add_argument("--schedule", default=None, metavar="PATH/CHUNK/MAX_FUSED[/SPLIT]",
                    help="install this apply schedule instead of tuning (e.g. mfma/32/3; "
                         "fixes the launches for profiling)")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint apply v = K^* h instead (1-D workloads)")
    ap.add_argument("--no-measured-peak", action="store_true",
                    help="skip the measured copy / MFMA-loop peaks in the roofline")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 256 MiB elementwise copy first (HBM counter calibration)")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-r", default="12",
                    help="order of every batched problem, or 'mlp' for the learned predictor")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "the IBF path here is single-GPU", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        _bench_batched(args)
        return
    if args.workload == "fio2d_256":
        _bench_2d(args)
        return
    if args.adjoint:
        _bench_adjoint(args)
        return

    import torch

    from paper_1605_03616_amd import ibf
    from paper_1605_03616_amd import inputs as I

    ibf.load()
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    P = _workload(args.workload, args.nrhs, args.precision)
    dt = torch.complex128 if P.precision == I.PREC_FP64 else torch.complex64
    print(f"[bench] workload {P.name} N={P.n} r={P.r} nrhs={P.nrhs} precision={P.precision}",
          file=sys.stderr, flush=True)

    pl = ibf.Plan.from_problem(P)
    torch.cuda.synchronize()
    # the first build in a process also loads the library's GPU code and warms
    # the allocator; it is reported apart, and the factorization is built
    # again from scratch for the build time
    t0 = time.perf_counter()
    pl.build()
    build_first_ms = (time.perf_counter() - t0) * 1e3
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
    tuning = None
    if args.schedule:        # a fixed schedule: no trial launches in a profile
        f = args.schedule.split("/")
        path, chunk, fused = f[0], int(f[1]), int(f[2])
        split = int(f[3]) if len(f) > 3 else 0
        pl.set_tuning(P.nrhs, path, chunk, fused, split)
        tuning = {"path": path, "chunk": chunk, "max_fused": fused, "split": split,
                  "fixed": True}
    elif not args.no_tune:   # schedule autotuner, before the timed region
        tuning = pl.tune(g, u)
        torch.cuda.synchronize()
        print(f"[bench] tuning: {tuning}", file=sys.stderr, flush=True)
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
        # BF16X2: the per-pair-rank stages multiply BF16 split products on the
        # bf16 MFMA (three bf16 products per algorithmic one, priced at the
        # published bf16 peak); the other stage kernels widen to FP32
        split = any(x[0] == "apply_stage_tight_split" for x in launches)
        bound, peak = ("hbm", HBM_PEAK_GBS) if P.nrhs < 64 else (
            "mfma", BF16_PEAK_TFS if split else FP32_PEAK_TFS)
    unit = "TFLOP/s" if bound == "mfma" else "GB/s"
    dom, roof, per_class = _roofline(launches, bound, peak, unit)
    sched = (f"{tuning['path']}/{tuning['chunk']}/{tuning['max_fused']}" if tuning
             else "default/0/0")
    if tuning and tuning.get("split"):
        sched += f"/{tuning['split']}"
    roof["traffic"] = _measured_traffic(P.name, sched, dom)
    if roof["traffic"] is not None:
        roof["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)"
    if not args.no_measured_peak and peak != BF16_PEAK_TFS:
        # the same bound measured on this device: a plain 1 GiB copy, or a loop
        # of the FP32 4x4x1 MFMA instruction the stage kernels issue
        what = ibf.PEAK_HBM_COPY if bound == "hbm" else ibf.PEAK_MFMA_F32
        mp = ibf.measure_peak(what)
        roof["measured_peak"] = round(mp, 3)
        roof["frac_measured"] = round(roof["achieved"] / mp, 4)
        roof["measured_peak_kind"] = ("plain device copy, read + write" if bound == "hbm"
                                      else "v_mfma_f32_4x4x1f32 loop, all CUs")

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
        "build_first_in_process_ms": round(build_first_ms, 3),
        "tuning": tuning,
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
        out["rel_err_vs_fp64"] = ibf.rel_error(u.to(torch.complex128), u64)[0]
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
        if P.precision == I.PREC_FP32:
            # the same workload with BF16X2 factors, beside the FP32 line: its
            # default schedule, error against the same FP64 IBF
            import dataclasses
            Pb = dataclasses.replace(P, precision=I.PREC_BF16X2)
            plb = ibf.Plan.from_problem(Pb)
            plb.build()
            ub = torch.empty_like(u)
            for _ in range(args.warmup):
                plb.apply(g, ub)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.steps):
                plb.apply(g, ub)
            e1.record(stream)
            torch.cuda.synchronize()
            msb = e0.elapsed_time(e1) / args.steps
            lb = plb.apply_profile(g, ub)
            out["bf16x2"] = {
                "value": round(P.n * P.nrhs / (msb * 1e-3) / 1e9, 4), "ms_per_step": round(msb, 5),
                "rel_err_vs_fp64": ibf.rel_error(ub.to(torch.complex128), u64)[0],
                "stage_kernel": max({x[0] for x in lb},
                                    key=lambda k: sum(x[1] for x in lb if x[0] == k)),
                "build_ms": round(plb.query()["build_ms"], 3)}
            plb.destroy()
        pl64.destroy()
        # the library's device FP64 direct product on sampled rows
        rows = I.error_rows(P.n)
        nchk = min(P.nrhs, 4)
        ud = ibf.dense_apply(P.phase, P.params,
                             torch.from_numpy(np.ascontiguousarray(P.x[rows])).cuda(),
                             torch.from_numpy(np.ascontiguousarray(P.xi)).cuda(),
                             g64[:nchk].contiguous())
        un = u[:nchk][:, torch.from_numpy(rows).cuda()].to(torch.complex128).contiguous()
        out["rel_err_vs_dense_sampled"] = ibf.rel_error(un, ud)[0]

    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = _cpu_baseline(P)
    pl.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
