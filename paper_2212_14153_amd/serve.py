"""Continuous-batching server for parameter-sweep simulations.

Requests (a simulation's parameters, its initial fiber and a step count) arrive over time.
The loop keeps one device batch (``Batch``, the C ABI's fpd_batch): whenever slots and HBM
budget allow, waiting requests are admitted between chunks of steps, so work that arrives
while others run overlaps with them on the device; finished simulations are read back and
released at once, which frees room for the next ones.  Each result is bitwise the result of
the same simulation run alone (per-simulation arithmetic does not depend on the mix).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib


@dataclass
class Request:
    rid: int
    params: object                 # _lib.fpd_params
    R: np.ndarray                  # initial bead positions [N, 2]
    steps: int
    arrival: float                 # seconds since the server started
    admitted: float = float("nan")
    finished: float = float("nan")
    status: int = -1
    beads: np.ndarray = field(default=None)   # final R
    populations: np.ndarray = field(default=None)   # final f[9, ny, nx] (if asked for)
    sim_id: int = 0
    lane: int = 0                  # the server's batch that ran it

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def run_batches(batches, max_steps: int, slice_steps: int = 512):
    """Advance several batches (each on its own stream) at the same time, up to max_steps
    steps each: in rounds of at most slice_steps steps, every batch's launch is enqueued
    before the first wait, so the streams' work interleaves on the device (a launch of many
    steps would fill the queue before the next batch's).  Returns the steps each batch
    advanced."""
    total = [0] * len(batches)
    live = list(range(len(batches)))
    while live:
        launched = []
        try:
            for i in live:
                launched.append((i, batches[i].launch(min(slice_steps,
                                                          max_steps - total[i]))))
        finally:
            for i, _ in launched:
                batches[i].wait()
        for i, adv in launched:
            total[i] += adv
        live = [i for i, adv in launched if adv > 0 and total[i] < max_steps]
    return total



class Server:
    """Admission by slots and HBM footprint; chunked execution; read-back on completion.

    With lanes > 1 the budget and slots are split over that many device batches, each on
    its own stream, advanced together (one batch's latency-bound bead kernels overlap
    another's lattice kernel); a request goes to the lane with the fewest nodes admitted."""

    def __init__(self, storage: str, hbm_budget: int, max_slots: int, chunk: int = 200,
                 stream=None, launch=None, clock=time.perf_counter, batch=None,
                 read_populations: bool = False, lanes: int = 1):
        # `batch` may be any object with the Batch methods used below (try_add, launch,
        # wait, poll, beads, release, set_launch, close; populations if read_populations),
        # or a list of them (one per lane); by default the device batches of the C ABI.
        # read_populations: read every finished simulation's populations back too
        # (Request.populations).
        if batch is not None:
            self.batches = list(batch) if isinstance(batch, (list, tuple)) else [batch]
        else:
            lanes = max(1, int(lanes))
            # lane 0 on the caller's stream (if given), the others on streams of their own
            self.batches = [_lib.Batch(hbm_budget // lanes, max(1, max_slots // lanes),
                                       storage=storage, stream=stream if k == 0 else None)
                            for k in range(lanes)]
        self.batch = self.batches[0]
        self.load = [0] * len(self.batches)   # nodes admitted per lane
        if launch:
            for b in self.batches:
                b.set_launch(launch)
        self.chunk = int(chunk)
        self.read_populations = bool(read_populations)
        self.clock = clock
        self.t0 = None
        self.waiting = collections.deque()
        self.running = {}
        self.done = []

    def close(self):
        for b in self.batches:
            b.close()

    def now(self) -> float:
        return self.clock() - self.t0

    def _admit(self):
        while self.waiting:
            req = self.waiting[0]
            nodes = int(req.params.nx) * int(req.params.ny)
            sid = None
            for lane in sorted(range(len(self.batches)), key=lambda k: self.load[k]):
                sid = self.batches[lane].try_add(req.params, req.R, req.steps)
                if sid is not None:
                    break
            if sid is None:
                if not self.running:
                    raise RuntimeError(f"request {req.rid} does not fit an empty batch")
                break
            self.waiting.popleft()
            req.sim_id = sid
            req.lane = lane
            req.admitted = self.now()
            self.load[lane] += nodes
            self.running[(lane, sid)] = req

    def _collect(self):
        for lane, b in enumerate(self.batches):
            for sid, status in b.poll():
                req = self.running.pop((lane, sid))
                req.status = status
                if status == _lib.FPD_SIM_DONE:
                    req.beads = b.beads(sid)[0]
                    if self.read_populations:
                        req.populations = b.populations(sid)
                req.finished = self.now()
                b.release(sid)
                self.load[lane] -= int(req.params.nx) * int(req.params.ny)
                self.done.append(req)

    def serve(self, requests, idle_sleep: float = 1e-3):
        """Serve `requests` (sorted by arrival time, seconds from start) to completion;
        returns them with admission and finish times filled in."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        total = len(pending)
        self.t0 = self.clock()
        while len(self.done) < total:
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.waiting.append(pending.popleft())
            self._admit()
            if self.running:
                run_batches(self.batches, self.chunk, slice_steps=self.chunk)
                self._collect()
            elif pending:
                time.sleep(min(idle_sleep, max(0.0, pending[0].arrival - self.now())))
        return self.done


def summarize(reqs, warmup: int = 0) -> dict:
    """p50 / p99 time-to-result and throughput over the requests after the first `warmup`
    arrivals."""
    reqs = sorted(reqs, key=lambda r: r.arrival)[warmup:]
    lat = np.array([r.latency for r in reqs])
    t_first = min(r.arrival for r in reqs)
    t_last = max(r.finished for r in reqs)
    ok = sum(1 for r in reqs if r.status == _lib.FPD_SIM_DONE)
    return {
        "requests": len(reqs), "completed": ok,
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()), "sims_per_s": ok / (t_last - t_first),
        "span_s": t_last - t_first,
    }


def fifo_replay(arrivals, service_times) -> np.ndarray:
    """Finish-minus-arrival times of a single FIFO server with the given service times."""
    t = 0.0
    out = []
    for a, s in zip(arrivals, service_times):
        t = max(t, a) + s
        out.append(t - a)
    return np.array(out)
