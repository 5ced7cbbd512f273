"""Host checks of bench.py's contract (no GPU): one GPU only, the stored
HBM traffic figures belong to the current apply source, and a workload's
factor precision can be replaced for side-by-side runs."""
import hashlib
import importlib.util
import os
import subprocess
import sys

from paper_1605_03616_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr


def test_measured_traffic_matches_the_apply_source():
    b = _bench()
    with open(b.APPLY_SRC, "rb") as f:
        sha = hashlib.sha1(f.read()).hexdigest()
    assert b.MEASURED_TRAFFIC
    for key, (src_sha, kernel, rows) in b.MEASURED_TRAFFIC.items():
        assert src_sha == sha, f"traffic of {key} was measured on another apply source"
        assert kernel.startswith("apply_") and rows and all(len(r) == 3 for r in rows)


def test_precision_override_renames_the_workload():
    b = _bench()
    P = b._workload("fio1d_1k")
    Q = b._workload("fio1d_1k", precision="bf16x2")
    assert Q.precision == I.PREC_BF16X2 and Q.name.endswith("_bf16x2")
    assert Q.n == P.n and Q.r == P.r and (Q.g == P.g).all()
    R = b._workload("fio1d_1k", precision={I.PREC_FP64: "fp64", I.PREC_FP32: "fp32",
                                           I.PREC_BF16X2: "bf16x2"}[P.precision])
    assert R.name == P.name
