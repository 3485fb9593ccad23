"""The fiber-ends recorder (fpd_record_*) on the GPU against the oracle's trajectory:
each record is the end-to-end vector and centroid of every fiber of the state R^n at the
start of step n (FP64: 1e-11 lu), every `every` steps, in a ring of `capacity` records.
Graph replay, direct launches and batches record the same values."""

import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu


def expected(traj0, traj, fibers, steps_wanted):
    """Rows [n, (ex, ey, cx, cy) per fiber] of R^n from the oracle (traj[k] = R^{k+1})."""
    rows = []
    for n in steps_wanted:
        R = traj0 if n == 0 else traj[n - 1]
        L = len(R) // fibers
        row = [float(n)]
        for c in range(fibers):
            f = R[c * L:(c + 1) * L]
            row += [f[-1, 0] - f[0, 0], f[-1, 1] - f[0, 1], f[:, 0].mean(), f[:, 1].mean()]
        rows.append(row)
    return np.array(rows)


def run_oracle(w, steps):
    st = oracle.make_state(oracle.OracleParams.from_mapping(w.params()), w.init_flow, w.beads())
    R0 = st.R.copy()
    traj = oracle.run(st, steps, trajectory=True)
    return R0, traj


@pytest.mark.parametrize("every,capacity,steps", [(5, 1000, 300), (3, 7, 50), (1, 64, 64)])
def test_record_matches_oracle(every, capacity, steps):
    w = workloads.c1_small_fp64()
    print(f"[case] record every={every} cap={capacity}", flush=True)
    R0, traj = run_oracle(w, steps)
    with _lib.simulation_from_workload(w, storage="f64") as sim:
        sim.step(7)                       # recording starts at step 7
        sim.record_start(every, capacity)
        sim.step(steps - 7)
        rec = sim.record()
    taken = list(range(7, steps, every))
    exp = expected(R0, traj, 1, taken[-capacity:])
    assert rec.shape == exp.shape
    assert np.array_equal(rec[:, 0], exp[:, 0])
    assert np.abs(rec[:, 1:] - exp[:, 1:]).max() < 1e-11


def test_record_several_fibers_and_launch_paths():
    w = workloads.fiber_suspension(n_fibers=3, beads=4, nx=150, ny=60, radius=1.5,
                                   re_ps=2.0, kappa=0.5, u_wall=0.02, storage="f64", seed=4)
    print("[case] record several fibers", flush=True)
    R0, traj = run_oracle(w, 120)
    recs = []
    for flags in (0, _lib.FPD_FLAG_NO_GRAPH):
        with _lib.simulation_from_workload(w, storage="f64", flags=flags) as sim:
            sim.set_launch(dict(graph_chunk=8))
            sim.record_start(4, 100)
            sim.step(120)
            recs.append(sim.record())
    exp = expected(R0, traj, 3, range(0, 120, 4))
    assert recs[0].shape == (30, 13)
    assert np.abs(recs[0] - exp).max() < 1e-11
    assert np.array_equal(recs[0], recs[1])


def test_record_in_a_batch_equals_alone():
    ws = [workloads.c1_small_fp64().with_(storage="f32", theta0=t) for t in (0.3, 1.1)]
    print("[case] record batch", flush=True)
    alone = []
    for w in ws:
        with _lib.simulation_from_workload(w, storage="f32") as sim:
            sim.record_start(2, 500)
            sim.step(100)
            alone.append(sim.record())
    params = [_lib.params_from_mapping(w.params(), storage="f32") for w in ws]
    budget = sum(_lib.fpd_sim_footprint(p) for p in params) * 2
    with _lib.Batch(budget, 2, storage="f32") as b:
        ids = [b.add(p, w.beads(), 100) for p, w in zip(params, ws)]
        for sid in ids:
            b.record_start(sid, 2, 500)
        while b.run(32):
            pass
        for sid, r in zip(ids, alone):
            assert np.array_equal(b.record(sid), r)


def test_record_errors():
    w = workloads.c1_small_fp64().with_(n_beads=0)
    with _lib.simulation_from_workload(w, storage="f64") as sim:
        with pytest.raises(_lib.FpdError) as e:
            sim.record_start(1, 10)
        assert e.value.code == _lib.FPD_ESTATE
    w = workloads.c1_small_fp64()
    with _lib.simulation_from_workload(w, storage="f64") as sim:
        with pytest.raises(_lib.FpdError):
            sim.record()
        with pytest.raises(_lib.FpdError):
            sim.record_start(0, 10)
        sim.record_start(1, 4)
        sim.step(3)
        assert sim.record().shape == (3, 5)
        sim.record_stop()
        sim.step(2)
