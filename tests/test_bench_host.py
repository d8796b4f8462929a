"""Host-side checks of bench.py (no GPU): the byte model, the traffic table and
the refusal of several GPUs."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_step_byte_model_totals():
    """Per-family algorithmic bytes per site and step add up to (10N + 56)P with
    the fused row-inverse force + LB pass, (10N + 58)P with the two apart."""
    fused = ["advect_update", "prop_row", "prop_col", "density", "force_row_fwd", "force_col", "force_inv_lb"]
    apart = fused[:-1] + ["force_row_inv", "lb"]
    for N in (16, 32, 64):
        for P in (4, 8):
            assert sum(bench.step_bytes_per_site(k, N, P) for k in fused) == (10 * N + 56) * P, (N, P)
            assert sum(bench.step_bytes_per_site(k, N, P) for k in apart) == (10 * N + 58) * P, (N, P)
    assert bench.step_bytes_per_site("lb", 32, 4) == 92
    assert bench.step_bytes_per_site("nn_conv", 32, 4) is None


def test_measured_traffic_entries_match_sources():
    """Every traffic entry names existing kernel sources; the current sources hash to
    the recorded value (a kernel change must re-measure or drop the entry)."""
    for key, tr in bench.MEASURED_TRAFFIC.items():
        assert tr["bytes_per_launch"] > 0
        assert bench.kernel_source_sha256(tr["files"]) == tr["source_sha256"], key
        assert bench.measured_traffic(*key) == tr["bytes_per_launch"]
    assert bench.measured_traffic("cfg3", "lb") is None


def test_window_starts_at_an_exact_step_inside_the_run():
    """The timed window holds exactly K steps, starts on a fallback step at least W
    steps into the run, and ends inside the 2e4-step run whenever it fits."""
    for K, W in ((20, 5), (2000, 50), (1, 0), (50, 0), (19990, 5), (30000, 7), (777, 333)):
        s = bench.window_start(20000, K, W)
        assert s % bench.FALLBACK_EVERY == 0 and s >= W, (K, W, s)
        if K + W + bench.FALLBACK_EVERY <= 20000:
            assert s + K <= 20000 and s + K > 20000 - bench.FALLBACK_EVERY - K % bench.FALLBACK_EVERY, (K, W, s)
    assert bench.window_start(20000, 20, 5) == 19950
    assert bench.window_start(20000, 2000, 50) == 18000


def test_bad_step_counts_refused():
    for argv in (["--steps", "0"], ["--steps", "-30"], ["--warmup", "-1"]):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 2 and "must be" in r.stderr, argv


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and h["available"] >= 1


def test_cpu_baseline_legs_run():
    """Both legs of the oracle baseline run on a small workload (the single
    process and the side-by-side processes, one thread each)."""
    r = bench.cpu_baseline("cfg1", 0.2, max_procs=2)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] == min(2, bench.host_cpu()["available"])
    assert r["single_core"]["value"] > 0 and r["single_core"]["cores"] == 1


def test_peaks_and_flop_model():
    assert bench.HBM_PEAK_GBS == 8000.0 and bench.BF16_MFMA_PEAK_TFLOPS == 2500.0
    assert bench.NN_FLOPS_PER_SITE["nn_conv"] == 73728
    assert os.path.exists(bench.WEIGHTS)


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_fluid3d_byte_model():
    """Per site and step: 19 populations read and 19 written plus the 3 force
    components, in the storage precision."""
    from paper_1804_02883_amd import fluid3d_timing as ft
    assert ft.bytes_per_site(1) == 164 and ft.bytes_per_site(0) == 328
    assert bench.measured_traffic("fluid3d_256", "lb3") is not None


def test_fluid3d_cpu_baseline_runs():
    r = bench.fluid3d_cpu_baseline(seconds=0.2, n=16)
    assert r["kind"] == "oracle" and r["value"] > 0 and r["cores"] == 1


def test_densities3d_cpu_baseline_runs():
    r = bench.densities3d_cpu_baseline(seconds=0.1, n=8, N=4)
    assert r["kind"] == "oracle" and r["value"] > 0
