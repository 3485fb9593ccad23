"""The autotuner on the device: tuning a simulation leaves its state bitwise where it was
(checkpoint and restore), and the tuned shape gives the same results as any other."""
import numpy as np
import pytest

import workloads
from paper_2212_14153_amd import _lib, autotune

pytestmark = pytest.mark.gpu


def test_tune_simulation_restores_state(tmp_path, monkeypatch):
    monkeypatch.setenv("FPD_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    w = workloads.c1_small_fp64()
    print("[case] autotune restore c1 f32", flush=True)
    with _lib.simulation_from_workload(w, storage="f32") as sim, \
            _lib.simulation_from_workload(w, storage="f32") as ref:
        sim.step(10)
        ref.step(10)
        f0, R0 = sim.populations(), sim.beads()[0]
        best, table = autotune.tune_simulation(sim, "f32", w.nx * w.ny, steps=4, rounds=1,
                                               use_cache=False)
        assert table is not None and sim.get_launch().block_x == best["block_x"]
        assert sim.steps == 10
        assert np.array_equal(sim.populations(), f0)
        assert np.array_equal(sim.beads()[0], R0)
        sim.step(10)
        ref.step(10)
        assert np.array_equal(sim.populations(), ref.populations())
        assert np.array_equal(sim.beads()[0], ref.beads()[0])
