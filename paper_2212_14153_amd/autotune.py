"""Launch-shape autotuner for the fused lattice kernel (single simulations and batches).

Candidates are (block_x, block_y, rows_per_thread, xcd_remap) shapes.  Every candidate is
timed on the real workload for a few steps, in several interleaved rounds (so clock and
thermal drift hit all candidates alike), and the fastest minimum wins.  Results are cached
in JSON keyed by GPU architecture, storage format and problem-size class; the cache lives
at $FPD_AUTOTUNE_CACHE or ~/.cache/fpdlbm/autotune.json.
"""
from __future__ import annotations

import itertools
import json
import math
import os
import sys
import tempfile
import time

SHAPES = [(256, 1), (128, 2), (128, 1), (64, 4), (64, 2), (64, 1)]
CANDIDATES = [dict(block_x=bx, block_y=by, rows_per_thread=spt, xcd_remap=xr)
              for (bx, by), spt, xr in itertools.product(SHAPES, (1, 2), (2, 1))]


def cache_path() -> str:
    return os.environ.get("FPD_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "fpdlbm", "autotune.json")


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home is fine: tuning just is not remembered


def device_key() -> str:
    try:
        import torch
        p = torch.cuda.get_device_properties(0)
        return getattr(p, "gcnArchName", p.name)
    except Exception:
        return "unknown"


def size_class(nodes: int) -> str:
    return f"2^{int(math.log2(max(nodes, 1)))}"


def search(run, candidates=None, rounds: int = 3):
    """run(cfg) -> seconds for a fixed amount of work; returns (best_cfg, table)."""
    candidates = list(candidates or CANDIDATES)
    best_t = {i: float("inf") for i in range(len(candidates))}
    for _ in range(rounds):
        for i, cfg in enumerate(candidates):
            best_t[i] = min(best_t[i], run(cfg))
    order = sorted(best_t, key=best_t.get)
    table = [(candidates[i], best_t[i]) for i in order]
    return candidates[order[0]], table


def _log_cached(key: str, cfg: dict) -> None:
    print(f"[autotune] {key}: cached launch shape {cfg} applied (from {cache_path()})",
          file=sys.stderr, flush=True)


def tune_simulation(sim, storage: str, nodes: int, steps: int = 40, rounds: int = 3,
                    use_cache: bool = True, restore: bool = True):
    """Pick and apply the best launch shape for one simulation.  Timing steps the
    simulation (rounds x candidates x (steps + 2) steps); with restore (the default) its
    state is saved to a temporary checkpoint first and loaded back afterwards, so the
    simulation is where it was, bitwise; restore=False leaves it advanced."""
    key = f"sim|{device_key()}|{storage}|{size_class(nodes)}"
    cache = _load_cache()
    if use_cache and key in cache:
        sim.set_launch(cache[key]["cfg"])
        _log_cached(key, cache[key]["cfg"])
        return cache[key]["cfg"], None
    saved = sim.get_launch()
    ckpt = None
    if restore:
        fd, ckpt = tempfile.mkstemp(prefix="fpd_autotune_", suffix=".ckpt")
        os.close(fd)
        sim.save(ckpt)

    def run(cfg):
        sim.set_launch(cfg)
        sim.step(2)
        sim.sync()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        return time.perf_counter() - t0

    try:
        best, table = search(run, rounds=rounds)
    finally:
        if ckpt:
            sim.load(ckpt)
            os.remove(ckpt)
    sim.set_launch(dict(best, graph_chunk=saved.graph_chunk))
    cache[key] = {"cfg": best, "seconds": table[0][1], "steps": steps}
    _store_cache(cache)
    return best, table


def tune_batch(make_batch, storage: str, nodes: int, steps: int = 16, rounds: int = 2,
               use_cache: bool = True):
    """make_batch() -> a fresh Batch holding the workload to tune on (each candidate runs a
    few steps of it).  Returns the best shape; the caller applies it to its own batch."""
    key = f"batch|{device_key()}|{storage}|{size_class(nodes)}"
    cache = _load_cache()
    if use_cache and key in cache:
        _log_cached(key, cache[key]["cfg"])
        return cache[key]["cfg"], None
    b = make_batch()
    try:
        def run(cfg):
            b.set_launch(dict(cfg, graph_chunk=8))
            b.run(8)
            t0 = time.perf_counter()
            b.run(steps)
            return time.perf_counter() - t0

        best, table = search(run, rounds=rounds)
    finally:
        b.close()
    cache[key] = {"cfg": best, "seconds": table[0][1], "steps": steps}
    _store_cache(cache)
    return best, table
