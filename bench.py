#!/usr/bin/env python
"""Throughput of the FPD fiber time step on one MI355X (arXiv:2212.14153, Sec. II.C).

Default workload: the 8192 x 2048 (16.8M nodes) confined-Couette channel with a 40-bead
fiber of radius 4 (Re_ps = 5, K = 3.3), FP32 populations, 2000 steps.  One "step" is the
whole path: the fused pull-stream + MRT-collide lattice kernel (with phi/eta/force density
near the fiber) and the per-bead kernel (Eq. 5 reduction, Euler update, A_i, forces).

Prints ONE JSON line with MLUPS (whole step, inputs resident in HBM), the lattice kernel's
HBM roofline (algorithmic 18 * sizeof(population) bytes per node per step over its event
time) and a CPU baseline (the FP64 oracle on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E peak
BYTES_PER_VALUE = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}
KERNEL_SRC = os.path.join(ROOT, "paper_2212_14153_amd", "csrc", "fpd_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_kernel.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name, storage):
    import workloads
    if name == "c1":
        return workloads.c1_small_fp64().with_(storage=storage)
    if name == "c2":
        return workloads.c2_medium_fp32().with_(storage=storage)
    return workloads.c3_large(storage)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(storage, nodes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source and this storage; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("entries", {}).get(storage)
    if not ent or rec.get("kernel_sha") != kernel_hash() or ent.get("nodes") != nodes:
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(w, steps):
    import numpy as np  # noqa: F401
    import oracle
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, w.init_flow, w.beads())
    oracle.run(st, 1)                      # first step outside the timing (page-in)
    t0 = time.perf_counter()
    oracle.run(st, steps)
    dt = time.perf_counter() - t0
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        model = platform.processor()
    return {
        "value": w.nx * w.ny * steps / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
        "sample": f"{w.nx}x{w.ny} lattice with the {w.n_beads}-bead fiber, {steps} FP64 steps "
                  f"after one untimed step, single-threaded C oracle ({dt:.1f} s)",
        "cpu_model": model, "host_cpus": os.cpu_count(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_VALUE))
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3"])
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="", help="block_x,block_y,rows_per_thread,xcd_remap")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); independent simulations shard across GPUs with no exchange, and "
              "no multi-GPU figure is produced here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_14153_amd import _lib

    w = workload(args.workload, args.storage)
    nodes = w.nx * w.ny
    torch.cuda.init()
    stream = torch.cuda.Stream()
    log(f"workload {w.name}: {w.nx}x{w.ny}, {w.n_beads} beads, storage {args.storage}")
    sim = _lib.simulation_from_workload(w, storage=args.storage, stream=stream.cuda_stream)
    if args.launch:
        bx, by, spt, xr = (int(v) for v in args.launch.split(","))
        sim.set_launch(dict(block_x=bx, block_y=by, rows_per_thread=spt, xcd_remap=xr))
    cfg = sim.get_launch()

    copy_gbps = _lib.fpd_copy_probe(stream.cuda_stream, 1 << 30, 20)
    log(f"copy probe: {copy_gbps:.0f} GB/s (read + write)")

    # warm-up (also captures the replay graphs)
    sim.step(args.warmup)
    sim.sync()
    torch.cuda.synchronize()

    # timed region: production path (graph replay), whole step
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    e1.synchronize()
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    mlups = nodes / (ms_step * 1e-3) / 1e6
    log(f"graph replay: {ms_step * 1e3:.1f} us/step, {mlups:.0f} MLUPS (wall {wall:.2f} s)")

    # same simulation, every kernel bracketed by events on its stream
    sim.set_flags(_lib.FPD_FLAG_TIME_KERNELS)
    sim.reset_kernel_times()
    e2 = torch.cuda.Event(enable_timing=True)
    e3 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e2.record(stream)
    sim.step(args.steps)
    e3.record(stream)
    e3.synchronize()
    sim.sync()
    ms_lat, n_lat, ms_bead, n_bead = sim.kernel_times()
    sim.set_flags(0)
    ms_timed_step = e2.elapsed_time(e3) / args.steps
    lat_ms = ms_lat / max(n_lat, 1)
    bead_ms = ms_bead / max(n_bead, 1) if n_bead else 0.0
    bytes_alg = 18 * BYTES_PER_VALUE[args.storage] * nodes
    achieved = bytes_alg / (lat_ms * 1e-3) / 1e9
    log(f"lattice kernel {lat_ms * 1e3:.1f} us ({achieved:.0f} GB/s), bead kernel "
        f"{bead_ms * 1e3:.1f} us")
    flags, strain = sim.health()
    sim.close()

    traffic = measured_traffic(args.storage, nodes)
    out = {
        "metric": "MLUPS & % HBM roofline", "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "nodes": nodes,
                   "n_beads": w.n_beads, "radius": w.radius, "re_ps": w.re_ps,
                   "kappa": w.kappa, "storage": args.storage, "parallelism": "single GPU",
                   "launch": cfg.__dict__},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "kernel": "step_kernel",
                     "bytes_per_launch_alg": bytes_alg, "avg_launch_ms": round(lat_ms, 5)},
        "bead_kernel_ms": round(bead_ms, 5),
        "ms_per_step_instrumented": round(ms_timed_step, 5),
        "copy_probe_gbps": round(copy_gbps, 1),
        "health_flags": flags, "max_bond_strain": strain,
    }
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle, {args.cpu_steps} steps of {w.name} in FP64")
        out["cpu_baseline"] = cpu_baseline(w.with_(storage="f64"), args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
