"""Host logic of bench.py: the one-GPU guard and the roofline bound choice
(a contraction is MFMA-bound when its flops per byte reach the ridge of its
dtype, peak flops / HBM bandwidth; every other class is HBM-bound)."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def _rec(ms, flops, nbytes, launches=1):
    return {"ms": ms, "flops": flops, "bytes": nbytes, "launches": launches}


def test_fp64_contraction_above_the_ridge_is_mfma_bound(bench):
    r = bench.roofline({"inner_products": _rec(1.0, 20e9, 1e9)}, 1)    # 20 flop/B > 9.8
    assert (r["bound"], r["unit"], r["peak"]) == ("mfma", "TFLOP/s", bench.PEAK["fp64_tflops"])
    assert r["achieved"] == pytest.approx(20.0)                       # 20 GFLOP in 1 ms
    assert r["frac"] == pytest.approx(20.0 / 78.6, abs=1e-5)


def test_fp64_contraction_below_the_ridge_is_hbm_bound(bench):
    r = bench.roofline({"inner_products": _rec(1.0, 5e9, 1e9)}, 1)     # 5 flop/B < 9.8
    assert (r["bound"], r["unit"], r["peak"]) == ("hbm", "GB/s", 8000.0)
    assert r["achieved"] == pytest.approx(1000.0)                     # 1 GB in 1 ms


def test_bf16_classes_use_the_bf16_ridge(bench):
    # 100 flop/B is far above the FP64 ridge but below BF16's 2500 / 8 = 312.5
    assert bench.roofline({"inner_products_bf16": _rec(1.0, 100e9, 1e9)}, 1)["bound"] == "hbm"
    r = bench.roofline({"sketch_bf16": _rec(1.0, 400e9, 1e9)}, 1)
    assert r["bound"] == "mfma" and r["peak"] == bench.PEAK["bf16_tflops"]


def test_latency_class_is_never_mfma_bound_and_the_largest_total_wins(bench):
    prof = {"sample_qrcp": _rec(5.0, 1e12, 1e6, launches=10),
            "inner_products": _rec(1.0, 20e9, 1e9)}
    r = bench.roofline(prof, 2)
    assert r["kernel"] == "sample_qrcp" and r["bound"] == "hbm"
    assert r["launches_per_step"] == 5 and r["avg_launch_us"] == 500.0
    assert r["achieved"] == pytest.approx(0.2)                        # 1 MB in 5 ms


def test_traffic_only_for_known_classes(bench):
    assert bench.measured_traffic("rqrcp_fp64_8000x8000_gauss", "omega11") is None
    assert bench.measured_traffic("no_such_workload", "sample_qrcp") is None
