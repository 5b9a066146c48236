"""Host logic of bench.py: which mixed policy the ventricle line reports, the sweep-rate and
roofline arithmetic, the traffic lookup and the one-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def run(its):
    return {"iterations": its}


@pytest.mark.parametrize("f32_its,err,met", [
    (343, 3e-12, True),      # fewer iterations, solution at the oracle's
    (350, 3e-12, True),      # FP64 + 2
    (351, 3e-12, False),     # FP64 + 3
    (343, 2e-6, False),      # the sample solution too far from the oracle's
    (350, None, True),       # no sample solved: the iteration bound alone
])
def test_mixed_contract(f32_its, err, met):
    e = None if err is None else {"mixed_f32fact_levels3": err}
    c = bench.mixed_contract(run(f32_its), run(348), e)
    assert c["met"] is met
    assert c["max_extra"] == 2 and c["max_error"] == 1e-6 and c["fp64_iterations"] == 348


def test_mixed_contract_needs_both_runs():
    assert bench.mixed_contract(None, run(348), None) is None
    assert bench.mixed_contract(run(343), {}, None) is None


def test_sweep_rate():
    r = {"breakdown": {"gj_interior": {"ms_per_step": 100.0, "flops": 6e12},
                       "gj_interface": {"ms_per_step": 20.0, "flops": 1e12},
                       "apply_whole": {"ms_per_step": 800.0, "flops": 0.0}}}
    f32 = bench.sweep_rate(r, "mixed_f32fact")
    assert f32["achieved_tflops"] == pytest.approx(7e12 / 0.12 / 1e12)
    assert f32["peak_tflops"] == bench.FP32_MFMA_PEAK_TFLOPS
    assert f32["frac"] == pytest.approx(f32["achieved_tflops"] / 157.3)
    assert f32["per_family_tflops"]["gj_interior"] == pytest.approx(60.0)
    assert bench.sweep_rate(r, "mixed")["peak_tflops"] == bench.FP64_PEAK_TFLOPS


def test_roofline_bound_and_rate():
    # 10 launches of 1 ms moving 5 GB each: HBM-bound, 5 TB/s
    hbm = bench.roofline({"ms": 10.0, "launches": 10, "bytes": 5e10, "flops": 1e9}, "no_such_family", "none")
    assert hbm["bound"] == "hbm" and hbm["achieved"] == pytest.approx(5000.0)
    assert hbm["frac"] == pytest.approx(5000.0 / 8000.0) and hbm["traffic"] is None
    # 2 launches of 1 ms with 40 GFLOP on 1 GB each: matrix-core bound, 40 TFLOP/s
    mf = bench.roofline({"ms": 2.0, "launches": 2, "bytes": 2e9, "flops": 8e10}, "no_such_family", "none")
    assert mf["bound"] == "mfma" and mf["achieved"] == pytest.approx(40.0)


def test_traffic_lookup_is_keyed_by_family_and_sources():
    assert bench.measured_traffic("no_such_family", "ventricle_1M") is None
    assert bench.measured_traffic("apply_H_average", "no_such_workload") is None
    h = bench.kernel_source_hash()
    assert len(h) == 64 and h == bench.kernel_source_hash()


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
