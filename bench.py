#!/usr/bin/env python
"""Throughput of the FPD fiber time step on one MI355X (arXiv:2212.14153, Sec. II.C).

Default workload: the 8192 x 2048 (16.8M nodes) confined-Couette channel with a 40-bead
fiber of radius 4 (Re_ps = 5, K = 3.3), FP32 populations.  One "step" is the whole path:
the fused pull-stream + MRT-collide lattice kernel (with phi/eta/force density near the
fiber) and the per-bead kernel (Eq. 5 reduction, Euler update, A_i, forces).  The timed
steps replay captured graphs (the chunk divides the timed step count; the graph is captured
before the timing starts).

Prints ONE JSON line with MLUPS (whole step, inputs resident in HBM), the lattice kernel's
HBM roofline (algorithmic 18 * sizeof(population) bytes per node per step over its
dispatch-stamped duration) and a CPU baseline (the FP64 oracle on a bounded sample of the
same workload).  Bounded runs of the other configurations are added as keys of the same
line (skip them with --no-extras):
  c2          the 1024 x 256 channel with the 20-bead fiber, FP32: MLUPS and effective GB/s
              (its two 9.4 MB buffers stay in the 256 MB Infinity Cache: not an HBM figure);
  sweep_c4    256 parameter-sweep simulations (128x64 .. 1024x512, 5-30 beads) advanced
              together by the batch kernels with autotuned tiles, against the plain path
              (a seeded random sample of them run one at a time, per-step launches, no
              graph, measured);
  serve_c5    Poisson arrivals of sweep simulations (20k steps each, FP16 deviation
              storage) served with continuous batching, at 50 requests/s and at 0.8 of the
              measured capacity: p50/p99 time-to-result and sims/s, against a measured
              first-in-first-out server of single simulations on the same arrivals;
  cpu_baseline_set  the oracle on C1 (1000 steps), C2 (1000 steps) and C3 in FP64 (20 steps).

Other modes (each prints one JSON line):
  --mode batch   the full C4 sweep (256 simulations, 20k steps each) against the plain path;
  --mode serve   the full C5 run (1000 requests after 100 warm-up at 50/s) against a
                 measured FIFO server of single simulations on a prefix of the arrivals;
  --mode particle  the driven-particle benchmark of Sec. III.B (periodic box, H = 10 d,
                 d = 20) swept over 64 driving forces in one batch (90k steps): C_d(Re_p), eps_v,
                 the diffuse-interface drag, and throughput;
  --mode sandwich  the Couette sandwich of Sec. III.A (H = 200, Re = 0.1) over a grid of
                 viscosity ratios and interface widths: steady-profile errors against
                 Eq. (13) and the exact smooth solution;
  --mode shapes  the shape diagrams of Sec. IV.C (K x C at Re_ps = 1.5, Re_ps x C at
                 K = 3.3e-5, and the stuck cases of rigid and slightly flexible fibers) as
                 recorded runs in two batches on two streams advanced together, each run
                 classified from its fiber-ends record.
"""
from __future__ import annotations

import argparse
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_kernel.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name, storage):
    import workloads
    if name == "c1":
        return workloads.c1_small_fp64().with_(storage=storage)
    if name == "c2":
        return workloads.c2_medium_fp32().with_(storage=storage)
    if name == "suspension":   # 25 fibers of 10 beads with C3's fiber and flow parameters
        return workloads.fiber_suspension(n_fibers=25, beads=10, nx=8192, ny=2048,
                                          radius=4.0, re_ps=5.0, kappa=3.3, u_wall=0.01,
                                          storage=storage)
    return workloads.c3_large(storage)


def kernel_hash() -> str:
    from paper_2212_14153_amd.profsum import kernel_source_hash
    return kernel_source_hash()


def measured_traffic(storage, nodes, workload, kernel="step_kernel"):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken
    on the current kernel source, this storage, this workload and these kernels; else
    None."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    ent = rec.get("entries", {}).get(storage)
    if (not ent or rec.get("kernel_sha") != kernel_hash() or ent.get("nodes") != nodes
            or ent.get("workload") != workload or ent.get("kernel") != kernel):
        return None
    return ent.get("bytes_per_launch")


def cpu_model() -> str:
    """The host CPU's full model name (the longer of lscpu's and /proc/cpuinfo's)."""
    names = []
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        names += [ln.split(":", 1)[1].strip() for ln in out.splitlines()
                  if ln.startswith("Model name")]
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            names += [ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")]
    except OSError:
        pass
    names.append(platform.processor())
    return max(names, key=len) if names else ""


def cpu_baseline(w, steps):
    """The oracle, single-threaded, on `steps` FP64 steps of workload w after one untimed
    step (page-in)."""
    import oracle
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, w.init_flow, w.beads())
    oracle.run(st, 1)
    t0 = time.perf_counter()
    oracle.run(st, steps)
    dt = time.perf_counter() - t0
    return {
        "value": round(w.nx * w.ny * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": 1,
        "kind": "oracle",
        "sample": f"{w.nx}x{w.ny} lattice with the {w.n_beads}-bead fiber, {steps} FP64 steps "
                  f"after one untimed step, single-threaded C oracle ({dt:.1f} s)",
        "seconds": round(dt, 2), "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
    }


def cpu_baseline_set(jobs):
    """cpu_baseline of several (label, workload, steps) at once, one thread each (the C
    oracle releases the interpreter lock; each run still uses one core)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    oracle.lib()
    oracle.inverse_moments([1.0] + [0.0] * 8)   # the oracle's lazy table, before threads
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        futs = {label: ex.submit(cpu_baseline, w, n) for label, w, n in jobs}
        return {label: f.result() for label, f in futs.items()}


def sweep_params(_lib, ws, storage, steps_override=None):
    return [_lib.params_from_mapping(w.params(), storage=storage) for w in ws]


def run_plain_path(_lib, ws, storage, steps, stream):
    """The plain path: one simulation at a time, one launch per kernel, no graph; the time of
    each simulation's steps (creation excluded) and its final beads."""
    times, finals = [], []
    for w in ws:
        sim = _lib.simulation_from_workload(w, storage=storage, stream=stream,
                                            flags=_lib.FPD_FLAG_NO_GRAPH)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        times.append(time.perf_counter() - t0)
        finals.append(sim.beads()[0])
        sim.close()
    return times, finals


def sweep_run(stream, storage, sims, steps, plain_sims, tune=True, seed=14153, batches=None):
    """C4: `sims` sweep simulations advanced together by the batch kernels (graph replay,
    launch shape from the autotuner), against the plain path measured on a seeded random
    sample of `plain_sims` of them.  `batches` (default: two for the two-byte formats, one
    otherwise) splits them over that many batches on as many streams, balanced by nodes.
    Returns the result keys."""
    import numpy as np
    import workloads
    from paper_2212_14153_amd import _lib, autotune, serve
    ws = workloads.sweep_sims(sims, seed=seed, steps=steps, storage=storage)
    params = sweep_params(_lib, ws, storage)
    nodes = sum(w.nx * w.ny for w in ws)
    budget = int(1.05 * sum(_lib.fpd_sim_footprint(p) for p in params)) + (1 << 26)
    log(f"sweep: {len(ws)} simulations, {nodes / 1e6:.1f}M nodes, {steps} steps each, "
        f"storage {storage}, {budget / 1e9:.2f} GB")

    def make_batch():
        b = _lib.Batch(budget, len(ws), storage=storage, stream=stream.cuda_stream)
        for p, w in zip(params, ws):
            b.add(p, w.beads(), 1 << 40)
        return b

    cfg = None
    if tune:
        cfg, _ = autotune.tune_batch(make_batch, storage, nodes)
        log(f"autotuned launch {cfg}")
    import torch
    nb = batches or (2 if storage in ("f16dev", "bf16dev") else 1)
    streams = [stream] + [torch.cuda.Stream() for _ in range(nb - 1)]
    bs = [_lib.Batch(budget, len(ws), storage=storage, stream=s.cuda_stream) for s in streams]
    load = [0] * nb
    ids = [None] * len(ws)
    for i in sorted(range(len(ws)), key=lambda i: -ws[i].nx * ws[i].ny):
        k = load.index(min(load))      # largest first onto the lighter batch
        load[k] += ws[i].nx * ws[i].ny
        ids[i] = (k, None)
    for b in bs:
        if cfg:
            b.set_launch(dict(cfg, graph_chunk=32))
    ids = [(k, bs[k].add(p, w.beads(), steps)) for (k, _), p, w in zip(ids, params, ws)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    finish = {}
    while len(finish) < len(ids):
        if max(serve.run_batches(bs, steps)) == 0:
            break
        t = time.perf_counter() - t0
        for k, b in enumerate(bs):
            for sid, st in b.poll():
                finish[(k, sid)] = (t, st)
    wall = time.perf_counter() - t0
    ok = sum(1 for t, st in finish.values() if st == _lib.FPD_SIM_DONE)
    rng = np.random.default_rng(seed + 1)
    pick = sorted(rng.choice(len(ws), size=min(plain_sims, len(ws)), replace=False).tolist())
    batch_R = [bs[ids[i][0]].beads(ids[i][1])[0] for i in pick]
    for b in bs:
        b.close()
    log(f"batched: {wall:.2f} s for {len(ids)} simulations ({ok} done); plain path on "
        f"{len(pick)} of them")
    out = {
        "workload": f"sweep of {len(ws)} simulations (seed {seed}), 128x64..1024x512, "
                    f"{steps} steps each, {storage}",
        "sims": len(ws), "steps": steps, "nodes_total": nodes, "launch": cfg, "batches": nb,
        "sims_per_s": round(ok / wall, 3), "seconds": round(wall, 3),
        "aggregate_mlups": round(nodes * steps / wall / 1e6, 1),
        "ms_per_batch_step": round(wall / steps * 1e3, 4),
    }
    if not pick:
        return out
    plain_t, plain_R = run_plain_path(_lib, [ws[i] for i in pick], storage, steps,
                                      stream.cuda_stream)
    plain_per_sim = float(np.mean(plain_t))
    # the sample's share of the sweep's work, to scale its time to all simulations
    frac = sum(ws[i].nx * ws[i].ny for i in pick) / nodes
    plain_all_s = float(np.sum(plain_t)) / frac
    diff = max(float(np.max(np.abs(a - c))) for a, c in zip(batch_R, plain_R))
    log(f"plain path: {plain_per_sim * 1e3:.1f} ms per simulation; batch == alone: "
        f"max bead difference {diff:.1e} lu")
    out.update({
        "plain_path": {"sample_sims": len(pick), "sample_seed": seed + 1,
                       "seconds_per_sim": round(plain_per_sim, 4),
                       "sims_per_s": round(len(pick) / float(np.sum(plain_t)), 3),
                       "all_sims_seconds_scaled_by_nodes": round(plain_all_s, 2)},
        "speedup_vs_plain": round(plain_all_s / wall, 2),
        "max_bead_diff_vs_plain_lu": diff,
    })
    return out


def plain_fifo(_lib, ws, arrivals, steps, storage, stream):
    """The plain path as a server, measured: requests in arrival order, one simulation at a
    time (created on arrival, per-step launches, no graph); time-to-result = finish -
    arrival.  Returns the latencies, the span from the first arrival to the last finish,
    and the final beads."""
    import numpy as np
    t0 = time.perf_counter()
    lat, finals = [], []
    for w, a in zip(ws, arrivals):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        sim = _lib.simulation_from_workload(w, storage=storage, stream=stream,
                                            flags=_lib.FPD_FLAG_NO_GRAPH)
        sim.step(steps)
        sim.sync()
        finals.append(sim.beads()[0])
        sim.close()
        lat.append(time.perf_counter() - t0 - a)
    span = time.perf_counter() - t0 - float(arrivals[0])
    return np.array(lat), span, finals


def serve_run(stream, storage, n_req, steps, rate, n_plain, warmup=0, slots=512, chunk=200,
              budget_gb=64, seed=50, lanes=1, tune=True):
    """C5 at one arrival rate: `n_req` Poisson arrivals of sweep simulations served with
    continuous batching, and the first `n_plain` of the same arrivals through the measured
    plain FIFO server.  Returns the result keys (p50 / p99 over the requests after
    `warmup`, and both paths over the same first n_plain requests)."""
    import numpy as np
    import workloads
    from paper_2212_14153_amd import _lib, serve
    ws = workloads.sweep_sims(n_req, seed=seed, steps=steps, storage=storage)
    arrivals = workloads.poisson_arrivals(n_req, rate=rate, seed=seed)
    params = sweep_params(_lib, ws, storage)
    reqs = [serve.Request(i, p, w.beads(), steps, float(t))
            for i, (p, w, t) in enumerate(zip(params, ws, arrivals))]
    log(f"serve: {n_req} requests at {rate:.1f}/s, {steps} steps each, storage {storage}")
    cfg = {}
    if tune:   # the batch launch shape, tuned on the requests' simulations (cached)
        from paper_2212_14153_amd import autotune
        budget = int(1.05 * sum(_lib.fpd_sim_footprint(p) for p in params)) + (1 << 26)

        def make_batch():
            b = _lib.Batch(budget, len(ws), storage=storage, stream=stream.cuda_stream)
            for p, w in zip(params, ws):
                b.add(p, w.beads(), 1 << 40)
            return b

        cfg, _ = autotune.tune_batch(make_batch, storage, sum(w.nx * w.ny for w in ws))
        log(f"serve: autotuned launch {cfg}")
    srv = serve.Server(storage, hbm_budget=budget_gb << 30, max_slots=slots, chunk=chunk,
                       stream=stream.cuda_stream, launch=dict(cfg, graph_chunk=32),
                       lanes=lanes)
    done = srv.serve(reqs)
    srv.close()
    summ = serve.summarize(done, warmup=warmup)
    by_id = {r.rid: r for r in done}
    head = [by_id[i] for i in range(n_plain)]
    lat_head = np.array([r.latency for r in head])
    log(f"served: p50 {summ['p50_s']:.2f} s, p99 {summ['p99_s']:.2f} s, "
        f"{summ['sims_per_s']:.1f} sims/s; plain FIFO on the first {n_plain}")
    lat_p, span_p, R_p = plain_fifo(_lib, ws[:n_plain], arrivals[:n_plain], steps, storage,
                                    stream.cuda_stream)
    diff = max(float(np.max(np.abs(r.beads - R)))
               for r, R in zip(head, R_p) if r.beads is not None)
    log(f"plain FIFO: p50 {np.percentile(lat_p, 50):.2f} s, p99 "
        f"{np.percentile(lat_p, 99):.2f} s, {n_plain / span_p:.2f} sims/s")
    pct = lambda a, q: round(float(np.percentile(a, q)), 3)  # noqa: E731
    return {
        "rate_per_s": round(rate, 3), "requests": n_req - warmup, "warmup": warmup,
        "lanes": lanes, "launch": cfg or None,
        "completed": summ["completed"], "sims_per_s": round(summ["sims_per_s"], 3),
        "p50_s": round(summ["p50_s"], 3), "p99_s": round(summ["p99_s"], 3),
        "mean_s": round(summ["mean_s"], 3), "span_s": round(summ["span_s"], 2),
        "first_requests": n_plain,
        "served_first": {"p50_s": pct(lat_head, 50), "p99_s": pct(lat_head, 99)},
        "plain_fifo_first": {"p50_s": pct(lat_p, 50), "p99_s": pct(lat_p, 99),
                             "sims_per_s": round(n_plain / span_p, 3),
                             "measured": "single simulations in arrival order, per-step "
                                         "launches, no graph"},
        "max_bead_diff_alone_vs_mix_lu": diff,
    }


def main_batch(args):
    import torch
    torch.cuda.init()
    stream = torch.cuda.Stream()
    r = sweep_run(stream, args.storage, args.sims, args.sweep_steps, args.plain_sims,
                  tune=not args.no_autotune, batches=args.sweep_batches or None)
    out = {
        "metric": "batched sims/s", "value": r["sims_per_s"], "unit": "sims/s",
        "n_gpus": 1, "steps": args.sweep_steps, "warmup": 0,
        "ms_per_step": r["ms_per_batch_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": r["workload"], "nodes_total": r["nodes_total"],
                   "launch": r["launch"], "parallelism": "single GPU"},
    }
    out.update({k: v for k, v in r.items() if k not in ("workload", "launch")})
    print(json.dumps(out), flush=True)


def main_serve(args):
    import torch
    torch.cuda.init()
    stream = torch.cuda.Stream()
    storage = args.storage if args.storage in ("f16dev", "bf16dev") else "f16dev"
    r = serve_run(stream, storage, args.requests + args.serve_warmup, args.sweep_steps,
                  args.rate, args.plain_requests, warmup=args.serve_warmup, slots=args.slots,
                  chunk=args.chunk, budget_gb=args.hbm_budget_gb, lanes=args.serve_lanes)
    out = {
        "metric": "served sims/s at p50/p99 time-to-result", "value": r["sims_per_s"],
        "unit": "sims/s", "n_gpus": 1, "steps": args.sweep_steps, "warmup": args.serve_warmup,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": storage, "data": "synthetic",
        "config": {"workload": f"Poisson {args.rate}/s sweep requests (seed 50), "
                               f"{args.sweep_steps} steps", "requests": args.requests,
                   "chunk": args.chunk, "slots": args.slots,
                   "hbm_budget_gb": args.hbm_budget_gb, "parallelism": "single GPU"},
    }
    out.update(r)
    print(json.dumps(out), flush=True)


def main_particle(args):
    """The driven-particle benchmark of Sec. III.B as a batched sweep over the driving
    force: a disk of diameter d = 20 lattice units (dx = d / 20) in a periodic box of side
    H = 10 d, interface xi = d / 8, r_eta = 50, pushed by F0 with the balancing body
    force; after a fixed number of steps, C_d (Eq. 16, |F_d| = F0 at steady state), Re_p,
    eps_v (Eq. 15) and the diffuse-interface drag of Eq. (17) for every force."""
    import numpy as np
    import torch
    import workloads
    from paper_2212_14153_amd import _lib, serve
    torch.cuda.init()
    stream = torch.cuda.Stream()
    storage = args.storage
    d, n, xi, nu = 20.0, 200, 2.5, 1.0 / 6.0
    forces = np.geomspace(args.f_min, args.f_max, args.particles)
    ws = [workloads.driven_particle(n=n, radius=d / 2, xi=xi, force=float(F), nu_f=nu,
                                    eta_ratio=50.0, storage=storage, steps=args.particle_steps)
          for F in forces]
    params = sweep_params(_lib, ws, storage)
    nodes = sum(w.nx * w.ny for w in ws)
    budget = int(1.05 * sum(_lib.fpd_sim_footprint(p) for p in params)) + (1 << 26)
    log(f"particle sweep: {len(ws)} boxes of {n}x{n}, F0 {forces[0]:.2e}..{forces[-1]:.2e}, "
        f"{args.particle_steps} steps, storage {storage}")
    # the boxes split over args.particle_batches batches on as many streams, advanced
    # together (one batch's bead kernel overlaps another's lattice kernel)
    nb = max(1, min(args.particle_batches, len(ws)))
    streams = [stream] + [torch.cuda.Stream() for _ in range(nb - 1)]
    batches = [_lib.Batch(budget, len(ws), storage=storage, stream=s.cuda_stream)
               for s in streams]
    placed = [(batches[i % nb], batches[i % nb].add(p, w.beads(), args.particle_steps))
              for i, (p, w) in enumerate(zip(params, ws))]
    half = args.particle_steps * 2 // 3

    def advance(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < n:
            adv = max(serve.run_batches(batches, n - done))
            if adv == 0:
                break
            done += adv
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3

    ms_first = advance(half)
    mid = [b.particle_stats(i) for b, i in placed]
    ms_total = ms_first + advance(args.particle_steps - half)
    end = [b.particle_stats(i) for b, i in placed]
    health = [b.info(i) for b, i in placed]
    for b in batches:
        b.close()
    curve = []
    for F, s0, s1, (steps_done, status, hflags) in zip(forces, mid, end, health):
        V0 = s1["V0x"]
        drag = -(s1["Fvisc_x"] + s1["Fpres_x"])
        curve.append({
            "F0": float(F), "V0": V0, "Re_p": V0 * d / nu,
            "C_d": float(F) / (0.5 * V0 * V0 * d),
            "eps_v_over_V0sq": s1["eps_v"] / (V0 * V0),
            "drag_eq17_over_F0": drag / float(F),
            "V0_change_last_third": abs(V0 - s0["V0x"]) / abs(V0),
            "status": int(status), "health": int(hflags)})
    steps = args.particle_steps
    mlups = nodes * steps / (ms_total * 1e-3) / 1e6
    bytes_alg = 18 * BYTES_PER_VALUE[storage] * nodes
    achieved = bytes_alg * steps / (ms_total * 1e-3) / 1e9
    out = {
        "metric": "driven-particle sweep MLUPS", "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": round(ms_total / steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": storage, "data": "synthetic",
        "config": {"workload": f"{len(ws)} driven particles, d = 20, H = 10 d, periodic "
                               f"{n}x{n}, xi = d/8, r_eta = 50", "nodes_total": nodes,
                   "batches": nb, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None,
                     "kernel": f"whole step of all boxes ({nb} batches on {nb} streams)",
                     "bytes_per_launch_alg": bytes_alg},
        "curve": curve,
    }
    if not args.no_cpu_baseline:
        import oracle
        w = ws[len(ws) // 2].with_(storage="f64")
        p = oracle.OracleParams.from_mapping(w.params())
        st = oracle.make_state(p, 0, w.beads())
        oracle.run(st, 1)
        t0 = time.perf_counter()
        oracle.run(st, args.cpu_steps * 10)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(n * n * args.cpu_steps * 10 / dt / 1e6, 3), "unit": "MLUPS",
            "cores": 1, "kind": "oracle",
            "sample": f"one {n}x{n} box, {args.cpu_steps * 10} FP64 steps ({dt:.1f} s)"}
    print(json.dumps(out), flush=True)


def main_sandwich(args):
    """The Couette sandwich benchmark of Sec. III.A as one batch: H = 200 (dx / H = 0.005),
    Re = 0.1, r_eta x r_xi grid; the steady v_x(y) against the sharp-interface solution
    (Eq. 13) and against the exact solution of the smooth profile (int 1/eta)."""
    import numpy as np
    import torch
    import workloads
    from paper_2212_14153_amd import _lib
    torch.cuda.init()
    stream = torch.cuda.Stream()
    storage = args.storage
    r_etas = [1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0]
    r_xis = [0.005, 0.01, 0.02, 0.05]
    H = 200
    ws = [workloads.sandwich(ny=H, nx=H, r_eta=r, r_xi=x, storage=storage,
                             steps=args.sandwich_steps)
          for r in r_etas for x in r_xis]
    params = sweep_params(_lib, ws, storage)
    nodes = sum(w.nx * w.ny for w in ws)
    budget = int(1.05 * sum(_lib.fpd_sim_footprint(p) for p in params)) + (1 << 26)
    log(f"sandwich sweep: {len(ws)} channels of {H}x{H}, {args.sandwich_steps} steps, {storage}")
    b = _lib.Batch(budget, len(ws), storage=storage, stream=stream.cuda_stream)
    ids = [b.add(p, w.beads(), args.sandwich_steps) for p, w in zip(params, ws)]
    for sid, w in zip(ids, ws):
        b.set_static_phi(sid, workloads.sandwich_phi(H, w.xi))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    while b.run(args.sandwich_steps):
        pass
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    rows = []
    y = np.arange(H) + 0.5
    yy = np.linspace(0, H, 400001)
    for sid, w in zip(ids, ws):
        u = b.fields(sid)[1][:, 0]
        U = w.u_wall
        inv = 1 / (w.nu_f * (1 + (w.eta_ratio - 1) * workloads.sandwich_phi_at(yy, H, w.xi)))
        cum = np.concatenate([[0], np.cumsum(0.5 * (inv[1:] + inv[:-1]) * np.diff(yy))])
        smooth = -U + 2 * U * np.interp(y, yy, cum) / cum[-1]
        sharp = np.clip(-U + 2 * U * (y - H / 3) / (H / 3), -U, U)
        rows.append({"r_eta": w.eta_ratio, "r_xi": w.xi / H,
                     "err_vs_sharp_eq13": float(np.abs(u - sharp).max() / (2 * U)),
                     "err_vs_smooth_exact": float(np.abs(u - smooth).max() / (2 * U))})
    b.close()
    steps = args.sandwich_steps
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    bytes_alg = 18 * BYTES_PER_VALUE[storage] * nodes
    achieved = bytes_alg * steps / (ms * 1e-3) / 1e9
    out = {
        "metric": "sandwich sweep MLUPS", "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round(ms / steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": storage,
        "data": "synthetic",
        "config": {"workload": f"{len(ws)} sandwich channels {H}x{H}, Re = 0.1, "
                               "r_eta 1-100 x r_xi 0.005-0.05", "nodes_total": nodes,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None, "kernel": "whole batch step",
                     "bytes_per_launch_alg": bytes_alg},
        "profiles": rows,
    }
    print(json.dumps(out), flush=True)


SHAPE_CONF = [0.3, 0.5, 0.6, 0.7, 0.8, 0.87]
SHAPE_KAPPA = [3.3e-5, 3.3e-4, 3.3e-3, 3.3e-2, 3.3e-1, 3.3, 33.0]
SHAPE_RE = [0.5, 1.5, 3.0, 4.5, 6.0, 7.5]


def shape_points():
    """(diagram, K, C, Re_ps) of every run: Fig. 10(a) K x C at Re_ps = 1.5, Fig. 10(b)
    Re_ps x C at K = 3.3e-5 (its Re_ps = 1.5 row is the K = 3.3e-5 row of (a)), and the
    stuck cases of Fig. 7 for K = 3.3 and 0.33 at (Re_ps, C) = (6, 0.5) and (6, 0.87)
    (their (1.5, 0.87) cases are in (a)), and the rigid fiber of Fig. 5 (K = 33): Re_ps
    from 0.5 to 4 at C = 0.2, and C = 0.2, 0.65, 0.75 at Re_ps = 1.5."""
    pts = [("a", k, c, 1.5) for k in SHAPE_KAPPA for c in SHAPE_CONF]
    pts += [("b", 3.3e-5, c, r) for r in SHAPE_RE if r != 1.5 for c in SHAPE_CONF]
    pts += [("stuck", k, c, r) for k in (3.3, 0.33) for r, c in ((6.0, 0.5), (6.0, 0.87))]
    pts += [("rigid", 33.0, 0.2, r) for r in (0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0)]
    pts += [("rigid", 33.0, c, 1.5) for c in (0.65, 0.75)]
    return pts


def main_shapes(args):
    """Shape diagrams of Sec. IV.C: N = 10 touching beads of d = 8 (r_c = 0.1), H = N d / C,
    L_x = 25 d, r_eta = 100, xi / d = 0.125, fiber flat at the centre, gamma = 1.5e-4 for
    every run; the fiber ends are recorded every 100 steps and each run is classified
    (stuck / Jeffery / S-turn / S-coiled) with its periods and stuck angle."""
    import torch
    import workloads
    from paper_2212_14153_amd import _lib, serve, tumbling
    torch.cuda.init()
    stream = torch.cuda.Stream()
    storage = args.storage
    steps, every, gamma = args.shape_steps, 100, 1.5e-4
    pts = shape_points()
    ws = [workloads.flexible_fiber(k, c, r, gamma=gamma, storage=storage, steps=steps)
          for _, k, c, r in pts]
    params = sweep_params(_lib, ws, storage)
    nodes = sum(w.nx * w.ny for w in ws)
    budget = int(1.05 * sum(_lib.fpd_sim_footprint(p) for p in params)) + (1 << 26)
    log(f"shape sweep: {len(ws)} channels, {nodes / 1e6:.2f}M nodes, {steps} steps "
        f"(gamma t = {gamma * steps:.0f}), storage {storage}")
    # the runs split over args.shape_batches batches on as many streams, advanced together
    # (one batch's bead and force kernels overlap another's lattice kernel)
    nb = max(1, min(args.shape_batches, len(ws)))
    streams = [stream] + [torch.cuda.Stream() for _ in range(nb - 1)]
    batches = [_lib.Batch(budget, len(ws), storage=storage, stream=s.cuda_stream)
               for s in streams]
    placed = []
    for i, (p, w) in enumerate(zip(params, ws)):
        b = batches[i % nb]
        sid = b.add(p, w.beads(), steps)
        b.record_start(sid, every, steps // every + 8)
        placed.append((b, sid))
    torch.cuda.synchronize()
    left, t0 = steps, time.perf_counter()
    while left > 0:
        adv = max(serve.run_batches(batches, min(left, 25000)))
        if adv == 0:
            break
        left -= adv
        log(f"  {steps - left} steps, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    rows = []
    for (diag, k, c, r), w, (b, sid) in zip(pts, ws, placed):
        done, status, hflags = b.info(sid)
        row = {"diagram": diag, "K": k, "C": round(w.confinement, 4), "Re_ps": r,
               "status": int(status), "health": int(hflags), "steps": int(done)}
        rec = b.record(sid) if status == _lib.FPD_SIM_DONE else []
        if len(rec) > 8:
            a = tumbling.analyse(rec, straight_length=(w.n_beads - 1) * w.l0, gamma=gamma)
            cross = tumbling.crossing_times(a["t"], a["theta"])
            row.update(orbit=tumbling.classify(a, gamma), turns=round(a["turns"], 3),
                       gT_first=round(gamma * cross[0], 2) if len(cross) else None,
                       gT_later=round(gamma * a["period"], 2) if len(cross) >= 2 else None,
                       L_min=round(a["L_min"], 3), L_mean=round(a["L_mean"], 3),
                       r_c_fit=round(a["r_c_fit"], 4),
                       final_angle_deg=round(tumbling.final_angle_deg(a), 1),
                       turn_sense="clockwise" if tumbling.turned_deg(a) < 0 else
                       "counter-clockwise")
        else:
            row["orbit"] = "failed"
        rows.append(row)
    for b in batches:
        b.close()
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    bytes_alg = 18 * BYTES_PER_VALUE[storage] * nodes
    achieved = bytes_alg * steps / (ms * 1e-3) / 1e9
    for row in rows:
        log(f"  {row['diagram']:5s} K={row['K']:<8.3g} C={row['C']:.3f} Re={row['Re_ps']:<4g} "
            f"{row['orbit']:9s} turns={row.get('turns')} gT1={row.get('gT_first')} "
            f"gT={row.get('gT_later')} Lmin={row.get('L_min')} rfit={row.get('r_c_fit')} "
            f"angle={row.get('final_angle_deg')} {row.get('turn_sense', '')}")
    out = {
        "metric": "shape sweep MLUPS", "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round(ms / steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": storage,
        "data": "synthetic",
        "config": {"workload": f"{len(ws)} confined-Couette fiber runs, N = 10, d = 8, "
                               f"H = N d / C, L_x = 25 d, r_eta = 100, xi = d / 8, "
                               f"gamma = {gamma:g}, recorded every {every} steps",
                   "nodes_total": nodes, "batches": nb, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": None,
                     "kernel": f"whole step of all runs ({nb} batches on {nb} streams)",
                     "bytes_per_launch_alg": bytes_alg},
        "runs": rows,
    }
    print(json.dumps(out), flush=True)


def choose_chunk(steps: int):
    """Graph chunk for `steps` timed steps: the largest even c <= 64 that divides steps (then
    every timed step runs in a replayed graph); for odd steps the largest even c <= 64 below
    steps (the last step then runs as direct launches); None below two steps."""
    for c in range(min(64, steps), 1, -1):
        if c % 2 == 0 and steps % c == 0:
            return c
    c = min(64, steps - steps % 2)
    return c if c >= 2 else None


def timed_path(steps: int, chunk):
    """What fpd_step does with `steps` steps and graph chunk `chunk`."""
    replays = steps // chunk if chunk and steps >= chunk else 0
    direct = steps - replays * (chunk or 0)
    return {"graph_chunk": chunk, "graph_replays": replays, "direct_steps": direct}


def time_steps(sim, stream, steps, warmup):
    """Warm-up, capture of the graph the timed steps replay, then `steps` timed steps
    (events on the simulation's stream); returns ms per step and the timed path."""
    import torch
    chunk = choose_chunk(steps)
    if chunk:
        sim.set_launch(dict(graph_chunk=chunk))
    sim.step(warmup)
    sim.sync()
    sim.capture(steps)          # outside the timed region
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    e1.synchronize()
    sim.sync()
    return e0.elapsed_time(e1) / steps, timed_path(steps, chunk)


def kernel_pass(sim, steps, warmup=4, flags=0):
    """The same number of steps again with every lattice and bead launch stamped by its own
    dispatch (FPD_FLAG_TIME_KERNELS added to `flags`: the steps split or whole as in the
    timed region), after `warmup` untimed steps in the same mode: average lattice-pass and
    bead kernel durations in ms.  The simulation's flags are `flags` afterwards."""
    from paper_2212_14153_amd import _lib
    sim.set_flags(_lib.FPD_FLAG_TIME_KERNELS | flags)
    sim.step(warmup)
    sim.sync()
    sim.reset_kernel_times()
    sim.step(steps)
    sim.sync()
    ms_lat, n_lat, ms_bead, n_bead = sim.kernel_times()
    sim.set_flags(flags)
    return ms_lat / max(n_lat, 1), (ms_bead / n_bead if n_bead else 0.0)


def c2_run(stream, steps=200, warmup=50, tune=True):
    """C2 (1024 x 256, 20 beads, FP32): MLUPS and the lattice kernel's effective GB/s.  Both
    population buffers (2 x 9.4 MB) fit the 256 MB Infinity Cache, so the rate measures the
    kernel on cache-resident data, not HBM.  The launch shape comes from the autotuner
    (cached; the simulation is restored after tuning): at this size narrower tiles than the
    large-lattice default pay."""
    from paper_2212_14153_amd import _lib, autotune
    w = workload("c2", "f32")
    nodes = w.nx * w.ny
    sim = _lib.simulation_from_workload(w, storage="f32", stream=stream.cuda_stream)
    cfg = None
    if tune:
        cfg, _ = autotune.tune_simulation(sim, "f32", nodes)
        log(f"c2: autotuned launch {cfg}")
    ms_step, path = time_steps(sim, stream, steps, warmup)
    lat_ms, bead_ms = kernel_pass(sim, steps)
    flags, _ = sim.health()
    sim.close()
    eff = 18 * 4 * nodes / (lat_ms * 1e-3) / 1e9
    log(f"c2: {ms_step * 1e3:.1f} us/step, {nodes / (ms_step * 1e3):.0f} MLUPS, lattice "
        f"kernel {lat_ms * 1e3:.1f} us = {eff:.0f} GB/s effective (MALL-resident)")
    return {"workload": w.name, "nx": w.nx, "ny": w.ny, "nodes": nodes, "steps": steps,
            "warmup": warmup, "dtype": "f32", "launch": cfg, "timed_path": path,
            "mlups": round(nodes / (ms_step * 1e-3) / 1e6, 1),
            "ms_per_step": round(ms_step, 5), "lattice_kernel_ms": round(lat_ms, 5),
            "bead_kernel_ms": round(bead_ms, 5),
            "effective_gbps": round(eff, 1),
            "effective_gbps_note": "18 x 4 B per node over the lattice kernel's duration; "
                                   "the 19 MB working set stays in the 256 MB Infinity "
                                   "Cache (MALL), so this is not an HBM rate",
            "health_flags": flags}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--storage", default="f32", choices=sorted(BYTES_PER_VALUE))
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "suspension"])
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline workload (no c2, sweep_c4, serve_c5 keys)")
    ap.add_argument("--launch", default="", help="block_x,block_y,rows_per_thread,xcd_remap")
    ap.add_argument("--no-split", action="store_true",
                    help="whole steps (FPD_FLAG_NO_SPLIT) in the timed region")
    ap.add_argument("--mode", default="plain",
                    choices=["plain", "batch", "serve", "particle", "sandwich", "shapes"])
    ap.add_argument("--shape-steps", type=int, default=400000)
    ap.add_argument("--shape-batches", type=int, default=2,
                    help="batches (streams) the shape runs are split over")
    ap.add_argument("--sandwich-steps", type=int, default=4000)
    ap.add_argument("--particles", type=int, default=64)
    ap.add_argument("--particle-steps", type=int, default=90000)
    ap.add_argument("--particle-batches", type=int, default=2,
                    help="batches (streams) the particle boxes are split over")
    ap.add_argument("--f-min", type=float, default=1e-4)
    ap.add_argument("--f-max", type=float, default=1e-1)
    ap.add_argument("--sims", type=int, default=256)
    ap.add_argument("--sweep-steps", type=int, default=20000)
    ap.add_argument("--plain-sims", type=int, default=32)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--sweep-batches", type=int, default=0,
                    help="batches (streams) the sweep is split over; 0: two for the "
                         "two-byte formats, one otherwise")
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--serve-warmup", type=int, default=100)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--plain-requests", type=int, default=40)
    ap.add_argument("--slots", type=int, default=512)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--serve-lanes", type=int, default=2,
                    help="batches (streams) the server spreads its requests over")
    ap.add_argument("--hbm-budget-gb", type=int, default=64)
    # sizes of the bounded runs added to the default line
    ap.add_argument("--x-sweep-sims", type=int, default=256)
    ap.add_argument("--x-sweep-steps", type=int, default=2000)
    ap.add_argument("--x-sweep-plain", type=int, default=64)
    ap.add_argument("--x-serve-requests", type=int, default=60)
    ap.add_argument("--x-serve-steps", type=int, default=20000)
    ap.add_argument("--x-serve-plain", type=int, default=24)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE "
              f"{world}); independent simulations shard across GPUs with no exchange, and "
              "no multi-GPU figure is produced here.", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batch":
        return main_batch(args)
    if args.mode == "serve":
        return main_serve(args)
    if args.mode == "particle":
        return main_particle(args)
    if args.mode == "sandwich":
        return main_sandwich(args)
    if args.mode == "shapes":
        return main_shapes(args)

    import torch
    from paper_2212_14153_amd import _lib

    t_start = time.perf_counter()
    w = workload(args.workload, args.storage)
    nodes = w.nx * w.ny
    torch.cuda.init()
    stream = torch.cuda.Stream()
    log(f"workload {w.name}: {w.nx}x{w.ny}, {w.n_beads} beads, storage {args.storage}")
    base_flags = _lib.FPD_FLAG_NO_SPLIT if args.no_split else 0
    sim = _lib.simulation_from_workload(w, storage=args.storage, stream=stream.cuda_stream,
                                        flags=base_flags)
    if args.launch:
        bx, by, spt, xr = (int(v) for v in args.launch.split(","))
        sim.set_launch(dict(block_x=bx, block_y=by, rows_per_thread=spt, xcd_remap=xr))

    copy_gbps = _lib.fpd_copy_probe(stream.cuda_stream, 1 << 30, 20)
    log(f"copy probe: {copy_gbps:.0f} GB/s (read + write)")

    # timed region: the production path (captured graphs replayed), whole step
    ms_step, path = time_steps(sim, stream, args.steps, args.warmup)
    path["split_steps"] = sim.split_active()
    cfg = sim.get_launch()
    mlups = nodes / (ms_step * 1e-3) / 1e6
    how = (f"{path['graph_replays']} graph replays of {path['graph_chunk']} steps"
           if path["graph_replays"] else "direct launches")
    if path["graph_replays"] and path["direct_steps"]:
        how += f" + {path['direct_steps']} direct steps"
    if path["split_steps"]:
        how += " (split steps)"
    log(f"{how}: {ms_step * 1e3:.1f} us/step, {mlups:.0f} MLUPS")

    # the same simulation, every lattice and bead launch stamped by its own dispatch (split
    # steps: the lattice pass from the earlier start to the later end of the fluid and
    # fiber kernels, beside each other)
    lat_ms, bead_ms = kernel_pass(sim, args.steps, flags=base_flags)
    lattice = "fluid_kernel+fiber_kernel" if path["split_steps"] else "step_kernel"
    bytes_alg = 18 * BYTES_PER_VALUE[args.storage] * nodes
    achieved = bytes_alg / (lat_ms * 1e-3) / 1e9
    log(f"lattice kernel {lat_ms * 1e3:.1f} us ({achieved:.0f} GB/s), bead kernel "
        f"{bead_ms * 1e3:.1f} us")
    flags, strain = sim.health()
    sim.close()

    traffic = measured_traffic(args.storage, nodes, args.workload, lattice)
    out = {
        "metric": "MLUPS & % HBM roofline", "value": round(mlups, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": w.name, "nx": w.nx, "ny": w.ny, "nodes": nodes,
                   "n_beads": w.n_beads, "radius": w.radius, "re_ps": w.re_ps,
                   "kappa": w.kappa, "storage": args.storage, "parallelism": "single GPU",
                   "launch": cfg.__dict__, "timed_path": path},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic, "kernel": lattice,
                     "bytes_per_launch_alg": bytes_alg, "avg_launch_ms": round(lat_ms, 5)},
        "bead_kernel_ms": round(bead_ms, 5),
        "copy_probe_gbps": round(copy_gbps, 1),
        "frac_of_copy_probe": round(achieved / copy_gbps, 4),
        "health_flags": flags, "max_bond_strain": strain,
    }
    if not args.no_extras and args.workload == "c3":
        out["c2"] = c2_run(stream)
        out["sweep_c4"] = sweep_run(stream, "f32", args.x_sweep_sims, args.x_sweep_steps,
                                    args.x_sweep_plain)
        at50 = serve_run(stream, "f16dev", args.x_serve_requests, args.x_serve_steps, 50.0,
                         args.x_serve_plain, lanes=args.serve_lanes)
        cap = at50["sims_per_s"]
        at08 = serve_run(stream, "f16dev", args.x_serve_requests, args.x_serve_steps,
                         0.8 * cap, args.x_serve_plain, lanes=args.serve_lanes)
        out["serve_c5"] = {"storage": "f16dev", "steps": args.x_serve_steps,
                           "lanes": args.serve_lanes,
                           "capacity_sims_per_s": cap, "at_50_per_s": at50,
                           "at_0.8_capacity": at08}
    if not args.no_cpu_baseline:
        head = f"{args.workload}_f64"
        jobs = [(head, w.with_(storage="f64"), args.cpu_steps)]
        if not args.no_extras and args.workload == "c3":
            jobs += [("c1_f64", workload("c1", "f64"), 1000),
                     ("c2_f64", workload("c2", "f64"), 1000)]
        log("cpu baseline: the oracle on " + ", ".join(f"{n} ({k} steps)" for n, _, k in jobs))
        res = cpu_baseline_set(jobs)
        out["cpu_baseline"] = res[head]
        if len(jobs) > 1:
            out["cpu_baseline_set"] = res
    else:
        out["cpu_baseline"] = None
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
