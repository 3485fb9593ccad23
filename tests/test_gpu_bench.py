"""The JSON line bench.py prints (a short run of the default workload, as a child process):
the fields a reader of the line relies on, and their consistency with each other."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*extra, timeout=110):
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *extra],
                         capture_output=True, text=True, timeout=timeout, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [ln for ln in out.stdout.splitlines() if ln.strip().startswith("{")]
    assert len(lines) == 1, out.stdout[-2000:]
    return json.loads(lines[0])


def test_default_bench_line():
    print("[case] bench.py --steps 20 --warmup 4 --no-cpu-baseline --no-extras", flush=True)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20",
                          "--warmup", "4", "--no-cpu-baseline", "--no-extras"],
                         capture_output=True, text=True, timeout=110, cwd=ROOT)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = [ln for ln in out.stdout.splitlines() if ln.strip().startswith("{")]
    assert len(lines) == 1, out.stdout[-2000:]
    d = json.loads(lines[0])
    assert d["metric"] == "MLUPS & % HBM roofline" and d["unit"] == "MLUPS"
    assert (d["n_gpus"], d["steps"], d["warmup"]) == (1, 20, 4)
    assert d["higher_is_better"] is True and d["data"] == "synthetic" and d["dtype"] == "f32"
    nodes = d["config"]["nodes"]
    assert nodes == 8192 * 2048 and "8192x2048" in d["config"]["workload"]
    # MLUPS of the whole step from its time per step
    assert d["value"] == pytest.approx(nodes / (d["ms_per_step"] * 1e-3) / 1e6, rel=2e-3)
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    # algorithmic bytes of the lattice kernel over its own measured duration
    assert r["bytes_per_launch_alg"] == 18 * 4 * nodes
    assert r["achieved"] == pytest.approx(r["bytes_per_launch_alg"] / r["avg_launch_ms"] / 1e6,
                                          rel=2e-3)
    assert 0.3 < r["frac"] < 1.0
    assert r["traffic"] is None or r["traffic"] >= r["bytes_per_launch_alg"]
    assert d["health_flags"] == 0
    # every timed step replayed a captured graph (the chunk divides the 20 steps), of split
    # steps (float32 with a 40-bead fiber on 8192 x 2048)
    assert d["config"]["timed_path"] == {"graph_chunk": 20, "graph_replays": 1,
                                         "direct_steps": 0, "split_steps": True}


def test_bench_line_extras_small():
    """The bounded runs of the other configurations, shrunk: their keys and consistency."""
    print("[case] bench.py extras (shrunk)", flush=True)
    d = run_bench("--steps", "8", "--warmup", "2", "--no-cpu-baseline",
                  "--x-sweep-sims", "6", "--x-sweep-steps", "100", "--x-sweep-plain", "2",
                  "--x-serve-requests", "5", "--x-serve-steps", "300", "--x-serve-plain", "2",
                  timeout=200)
    c2 = d["c2"]
    assert (c2["nx"], c2["ny"]) == (1024, 256) and c2["mlups"] > 0
    assert c2["effective_gbps"] == pytest.approx(72 * c2["nodes"] / c2["lattice_kernel_ms"]
                                                 / 1e6, rel=2e-3)
    s = d["sweep_c4"]
    assert s["sims"] == 6 and s["plain_path"]["sample_sims"] == 2
    assert s["max_bead_diff_vs_plain_lu"] == 0.0            # batched == alone, bitwise
    c5 = d["serve_c5"]
    for k in ("at_50_per_s", "at_0.8_capacity"):
        r = c5[k]
        assert r["completed"] == 5 and r["p99_s"] >= r["p50_s"] > 0
        assert r["plain_fifo_first"]["p99_s"] >= r["plain_fifo_first"]["p50_s"] > 0
        assert r["max_bead_diff_alone_vs_mix_lu"] == 0.0
    assert c5["at_0.8_capacity"]["rate_per_s"] == pytest.approx(
        0.8 * c5["capacity_sims_per_s"], rel=1e-3)
