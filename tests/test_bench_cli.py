"""Host-side behaviour of bench.py that needs no GPU: the one-GPU rule and
the traffic figure's guard on the kernel source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    summary = tmp_path / "summary.md"
    source = tmp_path / "kernels.hip"
    source.write_bytes(b"__global__ void k() {}\n")
    import hashlib
    digest = hashlib.sha256(source.read_bytes()).hexdigest()
    summary.write_text(f"- HBM bytes per launch: `1234.5`\n- kernel source sha256: `{digest}`\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(summary))
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(source))
    assert bench.measured_traffic("stencil_batched") == pytest.approx(1234.5)
    assert bench.measured_traffic("stencil_plain") is None       # another workload
    source.write_bytes(b"__global__ void k() { /* changed */ }\n")
    assert bench.measured_traffic("stencil_batched") is None     # the kernel changed since


def test_cpu_baseline_follows_the_cost_strata():
    # the CPU-baseline leg on a small space: every stratum the budget affords
    # is sampled, and the reported rate covers the whole space
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    from paper_2204_14242_amd import workloads as W
    k, hw, sp = W.stencil_plain()
    sp = dict(sp, domains=[(32, 32, 32)])
    n = 230
    evals = np.array([4 ** (5 + i % 4) for i in range(n)], dtype=np.float64)
    out = bench.cpu_baseline(k, hw, sp, evals, budget_s=2.0)
    assert out["kind"] == "oracle" and out["unit"] == "configs/s" and out["value"] > 0
    assert 1 <= out["cores"] <= 16 and out["cores"] <= out["nproc"]
    assert "4 cost strata" in out["sample"]
    assert out["checked_against_gpu"] == {"configs": 0, "identical": False}   # nothing given to check


def test_cpu_baseline_checks_the_given_records():
    # the sampled configurations' oracle records against records in canonical
    # order (here the oracle's own, standing in for the GPU's)
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    import oracle
    from paper_2204_14242_amd import workloads as W
    k, hw, sp = W.stencil_plain()
    sp = dict(sp, domains=[(32, 32, 32)])
    recs, _ = oracle.estimate(k, hw, sp, n_threads=4)
    evals = np.array([4 ** (5 + i % 4) for i in range(len(recs))], dtype=np.float64)
    out = bench.cpu_baseline(k, hw, sp, evals, budget_s=2.0, gpu_records=recs)
    assert out["checked_against_gpu"]["identical"] and out["checked_against_gpu"]["configs"] > 20
