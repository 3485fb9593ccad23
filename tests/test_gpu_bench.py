"""The JSON line bench.py prints (a short run of the default workload, as a child process):
the fields a reader of the line relies on, and their consistency with each other."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_default_bench_line():
    print("[case] bench.py --steps 20 --warmup 4 --no-cpu-baseline", flush=True)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20",
                          "--warmup", "4", "--no-cpu-baseline"], capture_output=True,
                         text=True, timeout=110, cwd=ROOT)
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
