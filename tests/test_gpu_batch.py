"""Batched simulations (kernels over (simulation, tile) and (simulation, bead) work items)
against the same simulations run alone through the single-simulation path."""
import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib, serve

pytestmark = pytest.mark.gpu


def small_sweep(storage, count=6, seed=7, steps=120):
    """Uneven lattices with fibers, drawn like the parameter sweep but small."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        ny = int(rng.integers(24, 70))
        n = int(rng.integers(2, 7))
        conf = float(rng.uniform(0.3, 0.7))
        l0 = conf * ny / n
        a = l0 / 2
        if a < 1.5:
            continue
        w = workloads.Workload(
            name=f"b{len(out)}", nx=int(rng.integers(30, 150)), ny=ny,
            u_wall=float(rng.uniform(0.005, 0.03)), nu_f=float(rng.uniform(0.03, 0.1)),
            eta_ratio=20.0, xi=1.0, n_beads=n, radius=a, l0=l0, k_s=0.05 * l0 * l0, k_b=1e-3,
            theta0=float(rng.uniform(0, np.pi)), cx=0.0, cy=ny / 2, steps=steps,
            storage=storage)
        w = w.with_(cx=w.nx / 2)
        if abs(np.sin(w.theta0)) * 0.5 * (n - 1) * l0 + a + 1.5 > ny / 2:
            w = w.with_(theta0=0.0)
        out.append(w)
    return out


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_batch_equals_each_simulation_alone(storage):
    ws = small_sweep(storage)
    print(f"[case] batch-vs-alone {storage} {[(w.nx, w.ny, w.n_beads) for w in ws]}", flush=True)
    # different step targets, so simulations leave the batch at different times
    targets = [120, 60, 120, 91, 30, 120]
    alone = []
    for w, t in zip(ws, targets):
        with _lib.simulation_from_workload(w, storage=storage) as sim:
            sim.step(t)
            alone.append((sim.populations(), sim.beads()[0]))
    with _lib.Batch(hbm_budget=1 << 33, max_slots=16, storage=storage) as b:
        b.set_launch(dict(graph_chunk=8))
        ids = [b.add(_lib.params_from_mapping(w.params(), storage=storage), w.beads(), t)
               for w, t in zip(ws, targets)]
        done = {}
        while len(done) < len(ids):
            adv = b.run(25)
            assert adv > 0
            for sid, st in b.poll():
                assert st == _lib.FPD_SIM_DONE
                done[sid] = (b.populations(sid), b.beads(sid)[0])
                steps, _, _ = b.info(sid)
                assert steps == targets[ids.index(sid)]
                b.release(sid)
        assert b.run(10) == 0
    for sid, (f, R) in zip(ids, alone):
        assert np.array_equal(done[sid][0], f)
        assert np.array_equal(done[sid][1], R)


def test_batch_matches_oracle():
    w = workloads.c1_small_fp64()
    print("[case] batch-oracle c1", flush=True)
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, 1, w.beads())
    oracle.run(st, 100)
    with _lib.Batch(hbm_budget=1 << 30, max_slots=4, storage="f64") as b:
        sid = b.add(_lib.params_from_mapping(w.params(), storage="f64"), w.beads(), 100)
        while b.run(1000):
            pass
        f = b.populations(sid)
        R = b.beads(sid)[0]
    assert np.max(np.abs(f - st.f) / st.f) <= 1e-12
    assert np.max(np.abs(R - st.R)) <= 1e-12


def test_admission_by_budget_and_slots():
    w = small_sweep("f32", count=1)[0]
    p = _lib.params_from_mapping(w.params(), storage="f32")
    need = _lib.fpd_sim_footprint(p)
    with _lib.Batch(hbm_budget=2 * need + need // 2, max_slots=8, storage="f32") as b:
        assert b.try_add(p, w.beads(), 10) is not None
        assert b.try_add(p, w.beads(), 10) is not None
        assert b.try_add(p, w.beads(), 10) is None          # budget
        assert b.stats()[1] == 2
    with _lib.Batch(hbm_budget=1 << 34, max_slots=1, storage="f32") as b:
        assert b.try_add(p, w.beads(), 10) is not None
        assert b.try_add(p, w.beads(), 10) is None          # slots
    with _lib.Batch(hbm_budget=1 << 34, max_slots=2, storage="f32") as b:
        with pytest.raises(_lib.FpdError):
            b.add(_lib.params_from_mapping(w.params(), storage="f64"), w.beads(), 10)


def test_unstable_simulation_is_evicted_and_others_continue():
    ws = small_sweep("f32", count=3, seed=3)
    print("[case] batch eviction", flush=True)
    with _lib.simulation_from_workload(ws[0], storage="f32") as sim:
        sim.step(80)
        ref = sim.populations()
    with _lib.Batch(hbm_budget=1 << 33, max_slots=8, storage="f32") as b:
        good = b.add(_lib.params_from_mapping(ws[0].params(), storage="f32"), ws[0].beads(), 80)
        # absurd stiffness: the fiber blows up within a few steps
        bad_p = _lib.params_from_mapping(ws[1].params(), storage="f32", k_s=1e6)
        bad = b.add(bad_p, ws[1].beads(), 80)
        status = {}
        while b.run(20):
            for sid, st in b.poll():
                status[sid] = st
        for sid, st in b.poll():
            status[sid] = st
        assert status[bad] == _lib.FPD_SIM_FAILED
        assert status[good] == _lib.FPD_SIM_DONE
        assert np.array_equal(b.populations(good), ref)


@pytest.mark.parametrize("bad", [dict(block_x=32), dict(block_y=3), dict(rows_per_thread=3),
                                 dict(xcd_remap=5), dict(graph_chunk=7)])
def test_invalid_batch_launch_is_refused_before_any_change(bad):
    ws = small_sweep("f32", count=2)
    print(f"[case] batch-launch {bad}", flush=True)
    with _lib.Batch(hbm_budget=1 << 33, max_slots=4, storage="f32") as empty:
        with pytest.raises(_lib.FpdError) as err:
            empty.set_launch(bad)
        assert err.value.code == _lib.FPD_EINVAL
    with _lib.Batch(hbm_budget=1 << 33, max_slots=4, storage="f32") as b:
        ids = [b.add(_lib.params_from_mapping(w.params(), storage="f32"), w.beads(), 20)
               for w in ws]
        with pytest.raises(_lib.FpdError) as err:
            b.set_launch(bad)
        assert err.value.code == _lib.FPD_EINVAL
        # the batch and its members keep the launch they had and still run
        assert b.run(20) == 20
        assert sorted(sid for sid, st in b.poll() if st == _lib.FPD_SIM_DONE) == sorted(ids)


def test_batches_on_two_streams_advance_together():
    """fpd_batch_launch / fpd_batch_wait: two batches on two streams advanced together give
    each simulation's result as run alone, bitwise; while a launch is pending the batch
    refuses other calls."""
    import torch
    ws = small_sweep("f32", seed=11)
    print(f"[case] two streams {[(w.nx, w.ny, w.n_beads) for w in ws]}", flush=True)
    targets = [120, 64, 120, 90, 32, 120]
    alone = []
    for w, t in zip(ws, targets):
        with _lib.simulation_from_workload(w) as sim:
            sim.step(t)
            alone.append(sim.beads()[0])
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    batches = [_lib.Batch(hbm_budget=1 << 33, max_slots=8, storage="f32",
                          stream=s.cuda_stream) for s in streams]
    try:
        where = {}
        for i, (w, t) in enumerate(zip(ws, targets)):
            b = batches[i % 2]
            b.set_launch(dict(graph_chunk=8))
            where[i] = (b, b.add(_lib.params_from_mapping(w.params()), w.beads(), t))
        # the pending guard: a read during a launch is refused, the launch still completes
        b0, sid0 = where[0]
        assert b0.launch(16) == 16
        with pytest.raises(_lib.FpdError):
            b0.beads(sid0)
        b0.wait()
        b0.wait()  # nothing pending: a no-op
        done = {}
        while len(done) < len(ws):
            adv = serve.run_batches(batches, 20)
            assert max(adv) > 0
            for i, (b, sid) in where.items():
                if i not in done and b.info(sid)[1] == _lib.FPD_SIM_DONE:
                    done[i] = b.beads(sid)[0]
        for i in range(len(ws)):
            assert np.array_equal(done[i], alone[i]), i
    finally:
        for b in batches:
            b.close()
