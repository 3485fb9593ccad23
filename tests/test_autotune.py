"""The launch-shape autotuner (host logic, no device): the search keeps each candidate's
fastest of several interleaved rounds, the winner is cached per device, storage and size
class and applied from the cache later, and tuning a simulation leaves its state as it was."""
import json
import types

import pytest

from paper_2212_14153_amd import autotune


class Clock:
    def __init__(self):
        self.t = 0.0

    def perf_counter(self):
        return self.t


def cost(cfg):
    """A made-up time per step for a launch shape (128x2, one row, no remap is fastest)."""
    return (abs(cfg["block_x"] - 128) / 64 + abs(cfg["block_y"] - 2) + cfg["rows_per_thread"]
            + (0.5 if cfg["xcd_remap"] == 1 else 0.0)) * 1e-3 + 1e-3


def test_search_takes_each_candidates_best_round():
    calls = []
    n = len(autotune.CANDIDATES)

    def run(cfg):
        # noise by (round, place in the round): each candidate meets every value, 0 once
        r, i = divmod(len(calls), n)
        calls.append(cfg)
        return cost(cfg) + [0.5, 0.0, 0.3][(r + i) % 3] * 1e-4

    best, table = autotune.search(run, rounds=3)
    assert len(calls) == 3 * n                                 # every candidate, every round
    assert calls[:n] == calls[n:2 * n] == autotune.CANDIDATES  # rounds interleave candidates
    assert best == dict(block_x=128, block_y=2, rows_per_thread=1, xcd_remap=2)
    times = [t for _, t in table]
    assert times == sorted(times)                              # fastest first
    best_t = dict((json.dumps(c, sort_keys=True), t) for c, t in table)
    for c in autotune.CANDIDATES:                              # minimum over its rounds
        assert best_t[json.dumps(c, sort_keys=True)] == pytest.approx(cost(c), abs=1e-12)


class FakeBatch:
    def __init__(self, clock):
        self.clock, self.cfg, self.closed = clock, None, False

    def set_launch(self, cfg):
        self.cfg = cfg

    def run(self, steps):
        self.clock.t += steps * cost(self.cfg)
        return steps

    def close(self):
        self.closed = True


def test_tune_batch_caches_and_reuses(tmp_path, monkeypatch, capsys):
    clock = Clock()
    monkeypatch.setattr(autotune, "time", types.SimpleNamespace(perf_counter=clock.perf_counter))
    monkeypatch.setenv("FPD_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    made = []

    def make():
        made.append(FakeBatch(clock))
        return made[-1]

    best, table = autotune.tune_batch(make, "f32", 1 << 20)
    assert best == dict(block_x=128, block_y=2, rows_per_thread=1, xcd_remap=2)
    assert table is not None and len(made) == 1 and made[0].closed
    cache = json.loads((tmp_path / "tune.json").read_text())
    key = f"batch|{autotune.device_key()}|f32|2^20"
    assert cache[key]["cfg"] == best
    # a second call of the same size class applies the cached shape without timing
    again, table2 = autotune.tune_batch(make, "f32", (1 << 20) + 5)
    assert again == best and table2 is None and len(made) == 1
    assert "cached launch shape" in capsys.readouterr().err
    # another storage or size class is tuned afresh
    autotune.tune_batch(make, "f16dev", 1 << 20)
    assert len(made) == 2


class FakeSim:
    """The Simulation methods the tuner uses; save / load keep the step count."""
    def __init__(self, clock):
        self.clock, self.steps = clock, 0
        self.cfg = dict(block_x=256, block_y=1, rows_per_thread=1, xcd_remap=2, graph_chunk=64)

    def get_launch(self):
        return types.SimpleNamespace(graph_chunk=self.cfg.get("graph_chunk", 64))

    def set_launch(self, cfg):
        self.cfg = dict(self.cfg, **cfg)

    def step(self, n):
        self.steps += n
        self.clock.t += n * cost(self.cfg)

    def sync(self):
        pass

    def save(self, path):
        with open(path, "w") as f:
            f.write(str(self.steps))

    def load(self, path):
        with open(path) as f:
            self.steps = int(f.read())


def test_tune_simulation_restores_the_state(tmp_path, monkeypatch):
    clock = Clock()
    monkeypatch.setattr(autotune, "time", types.SimpleNamespace(perf_counter=clock.perf_counter))
    monkeypatch.setenv("FPD_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sim = FakeSim(clock)
    sim.step(7)
    best, table = autotune.tune_simulation(sim, "f32", 4096)
    assert best == dict(block_x=128, block_y=2, rows_per_thread=1, xcd_remap=2)
    assert sim.steps == 7                                    # where it was before tuning
    assert sim.cfg["block_x"] == 128 and sim.cfg["graph_chunk"] == 64
    assert not list(tmp_path.glob("fpd_autotune_*"))         # the checkpoint is gone
    sim2 = FakeSim(clock)
    autotune.tune_simulation(sim2, "f16dev", 4096, restore=False)
    assert sim2.steps == 3 * len(autotune.CANDIDATES) * 42  # advanced when asked not to restore
