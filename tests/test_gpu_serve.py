"""Continuous batching on the GPU: requests arriving while others run are admitted as
slots free up (in one batch, or spread over two on two streams), and each result (bead
positions and every population) equals the same simulation run alone, bitwise."""
import numpy as np
import pytest

import workloads
from paper_2212_14153_amd import _lib, serve

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("storage,lanes", [("f16dev", 1), ("bf16dev", 1), ("f16dev", 2)])
def test_served_results_equal_alone(storage, lanes):
    print(f"[case] serve {storage} lanes={lanes}", flush=True)
    ws = [w.with_(storage=storage) for w in workloads.sweep_sims(10, seed=5, steps=300)]
    arrivals = np.linspace(0.0, 0.05, len(ws))
    reqs = [serve.Request(i, _lib.params_from_mapping(w.params(), storage=storage), w.beads(),
                          300 if i % 3 else 150, float(t))
            for i, (w, t) in enumerate(zip(ws, arrivals))]
    srv = serve.Server(storage, hbm_budget=1 << 34, max_slots=4, chunk=40,
                       launch=dict(graph_chunk=8), read_populations=True, lanes=lanes)
    done = srv.serve(reqs)
    srv.close()
    assert len(done) == len(reqs)
    assert all(r.status == _lib.FPD_SIM_DONE for r in done)
    assert {r.lane for r in done} == set(range(lanes))
    s = serve.summarize(done)
    assert s["p99_s"] >= s["p50_s"] > 0
    for r in done:
        with _lib.simulation_from_workload(ws[r.rid], storage=storage) as sim:
            sim.step(r.steps)
            assert np.array_equal(sim.beads()[0], r.beads)
            assert np.array_equal(sim.populations(), r.populations)   # the whole fluid too
