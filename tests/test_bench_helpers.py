"""Host-side helpers of bench.py (no GPU): argument defaults, the stored oracle
samples it compares with, the traffic record's applicability rules, and the
refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def parse(*argv):
    old = sys.argv
    sys.argv = ["bench.py", *argv]
    try:
        return bench.parse()
    finally:
        sys.argv = old


def test_defaults_are_the_headline_configuration():
    a = parse()
    assert a.gpus == 1 and a.steps == 5 and a.warmup == 1
    assert a.workload == "many_drops" and a.n is None and a.drops == 32 and a.tol == 1e-10
    assert a.coefficients == "density"
    assert "32 drops" in bench.layout_text(a)


@pytest.mark.parametrize("workload,n,drops,present", [
    ("many_drops", 512, 32, True), ("many_drops", 512, 16, False), ("many_drops", 256, 32, False),
    ("drop_film", 128, 32, True), ("spheroid_film", 256, 32, True), ("sphere", 32, 32, False)])
def test_stored_oracle_samples_are_found_for_their_workload_only(workload, n, drops, present):
    path = bench.golden_path(workload, n, drops)
    assert (path is not None) == present
    if path:
        assert os.path.basename(path) == f"{workload}{n}_oracle.txt"


def test_traffic_record_applies_to_its_kernels_and_size_only():
    assert bench.measured_traffic("mgp::k_resid<float, 1, false>", 512) is None
    known = {bench.kernel_symbol("sweep2", "mixed", "density"), bench.kernel_symbol("outer_update", "mixed", "density")}
    for k in bench.TRAFFIC["kernels"]:
        assert k in known
        assert bench.measured_traffic(k, 256) is None
    assert bench.TRAFFIC["fetch_scale"] > 0 and bench.TRAFFIC["write_scale"] > 0


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "single-GPU" in msg["error"]


def test_cpu_baseline_runs_the_whole_oracle_solve_and_reports_the_host():
    from paper_2605_30082_amd import workloads as W
    wl = W.make("sphere", 16)
    cpu = bench.cpu_baseline(wl, parse("--workload", "sphere", "--n", "16"), 9)
    assert cpu["kind"] == "oracle" and cpu["unit"] == "ms" and cpu["value"] > 0
    assert cpu["rel_res"] <= 1e-10 and 5 <= cpu["cycles"] <= 30
    assert cpu["cores"] >= 1 and cpu["single_thread_one_cycle_s"] > 0
    host = cpu["host"]
    assert host["logical_cpus_usable"] >= 1
    if cpu["peak_rss_gib"] is not None:
        assert cpu["peak_rss_gib"] >= cpu["rss_before_gib"] > 0
