"""bench.py as the driver runs it, and each of its workloads (subprocesses on the GPU)."""
import json
import os
import subprocess
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.gpu


def run_bench(args, timeout):
    t0 = time.perf_counter()
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args, cwd=ROOT, capture_output=True,
                       text=True, timeout=timeout)
    wall = time.perf_counter() - t0
    sys.stdout.write(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout[-2000:]
    return json.loads(lines[0]), wall


def test_driver_command():
    """python3 bench.py --gpus 1 --steps 20 --warmup 5: one JSON line with the
    contract's keys, the roofline and the CPU baseline, and a timed region that
    fits inside the process's wall time."""
    out, wall = run_bench(["--gpus", "1", "--steps", "20", "--warmup", "5"], 900)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in out, k
    assert out["steps"] == 20 and out["warmup"] == 5 and out["n_gpus"] == 1 and out["value"] > 0
    assert out["ms_per_step"] * out["steps"] / 1e3 < wall
    assert out["config"]["window_start"] % 50 == 0 and out["config"]["window_start"] >= 5
    assert out["config"]["window_exact_steps"] >= 1
    rl = out["roofline"]
    assert rl["bound"] in ("mfma", "hbm") and rl["achieved"] > 0 and 0 < rl["frac"] < 1
    assert abs(rl["frac"] - rl["achieved"] / rl["peak"]) < 1e-3
    cb = out["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["single_core"]["cores"] == 1
    assert cb["host"]["nproc"] >= 1
    # the plain path's kernels, each timed at its own start and end, fit in its step
    assert out["plain"]["kernel_sum_us_per_step"] <= 1.02 * 1e3 * out["plain"]["ms_per_step"]
    assert out["density_err"]["in_use"] <= 1e-3
    # the probes ran: the layer's ceilings order as matrix work <= work + stores
    cf = out["conv_floor"]
    assert 0 < cf["mfma"]["us"] <= cf["mfma_store"]["us"] and cf["store"]["us"] > 0, cf
    assert out["sync_costs"]["graph_node_gpu_us"] > 0


@pytest.mark.parametrize("wl", ["cfg2", "cfg3", "cfg5", "cfg4"])
def test_plain_workloads(wl):
    out, wall = run_bench(["--workload", wl, "--steps", "20", "--warmup", "5", "--no-cpu-baseline",
                           "--no-secondary"], 600)
    assert out["config"]["path"] == "plain" and out["config"]["workload"].startswith(wl)
    assert out["steps"] == 20 and out["value"] > 0 and out["roofline"]["bound"] == "hbm"
    assert out["ms_per_step"] * 20 / 1e3 < wall
    # the profiled launches are stream launches, each timed from its own start
    # to its end; at 1024 x 512 the kernels dominate and their sum fits in the
    # graph-replayed step, while on smaller grids each short kernel's timed
    # extent carries its launch's event work (cfg2: 250 us of kernels against
    # a 231 us step); the groups of a batch run as concurrent graph branches
    if wl == "cfg3":
        assert out["roofline"]["kernel_sum_us_per_step"] <= 1.05 * 1e3 * out["ms_per_step"]
    elif wl != "cfg4":
        assert out["roofline"]["kernel_sum_us_per_step"] <= 1.3 * 1e3 * out["ms_per_step"]


def test_surrogate_line_without_secondaries():
    out, _ = run_bench(["--steps", "100", "--warmup", "0", "--no-cpu-baseline", "--no-secondary"], 600)
    assert out["config"]["path"] == "surrogate" and out["steps"] == 100
    assert "plain_full_scale" not in out and "cpu_baseline" not in out
    assert out["speedup"] > 1.0
