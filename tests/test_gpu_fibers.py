"""Several fibers on the GPU (fibers of n_beads / n_chains consecutive beads, meeting
through the fluid and, when switched on, an excluded volume) against the oracle, through
the C ABI: populations and beads after coupled steps (FP64 1e-12 relative / 1e-11 lu, FP32
1e-5 / 1e-4 lu, the FP32 bound of the single-fiber runs), the forces read back at the
start, the point symmetry of a symmetric pair, bitwise launch-shape independence, and
batch equality."""

import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def small_suspension(storage, n_fibers=3, beads=4, seed=4):
    return workloads.fiber_suspension(n_fibers=n_fibers, beads=beads, nx=150, ny=60,
                                      radius=1.5, re_ps=2.0, kappa=0.5, u_wall=0.02,
                                      storage=storage, seed=seed)


@pytest.mark.parametrize("storage,tol_f,tol_r", [("f64", 1e-12, 1e-11), ("f32", 1e-5, 1e-4)])
def test_several_fibers_match_oracle(storage, tol_f, tol_r):
    w = small_suspension(storage)
    print(f"[case] suspension {storage}", flush=True)
    st = oracle.make_state(oracle.OracleParams.from_mapping(w.params()), 1, w.beads())
    oracle.run(st, 300)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.step(300)
        sim.sync()
        f = sim.populations()
        R = sim.beads()[0]
        flags, _ = sim.health()
    assert flags == 0
    assert rel_err(f, st.f) <= tol_f
    assert np.max(np.abs(R - st.R)) <= tol_r
    assert np.abs(R - w.beads()).max() > 1e-3      # the fibers move


def test_symmetric_pair_stays_point_symmetric():
    nx, ny, L = 64, 40, 4
    c = np.array([nx / 2, ny / 2])
    A = workloads.straight_fiber(L, 2.0, 0.5, c[0] - 12.0, c[1] + 5.0)
    B = 2 * c - A[::-1]
    w = workloads.Workload(name="pair", nx=nx, ny=ny, u_wall=0.01, nu_f=0.05, eta_ratio=20.0,
                           xi=1.0, n_beads=2 * L, radius=1.0, l0=2.0, k_s=0.3, k_b=2e-3,
                           theta0=0.0, cx=0.0, cy=0.0, steps=0, storage="f64", n_chains=2,
                           centres=((0, 0, 0), (0, 0, 0)))
    print("[case] symmetric pair", flush=True)
    p = _lib.params_from_mapping(w.params(), storage="f64")
    with _lib.Simulation(p) as sim:
        sim.init_fiber(np.concatenate([A, B]))
        sim.step(400)
        R = sim.beads()[0]
    assert np.abs(R[:L] + R[L:][::-1] - 2 * c).max() < 1e-10


def test_launch_shapes_are_bitwise_identical_with_several_fibers():
    w = small_suspension("f32", n_fibers=4, beads=3, seed=9)
    print("[case] suspension launch shapes", flush=True)
    outs = []
    for cfg in (dict(block_x=256, block_y=1, rows_per_thread=1),
                dict(block_x=64, block_y=4, rows_per_thread=2),
                dict(block_x=128, block_y=2, rows_per_thread=4)):
        with _lib.simulation_from_workload(w, storage="f32") as sim:
            sim.set_launch(cfg)
            sim.step(64)
            outs.append((sim.populations(), sim.beads()[0]))
    for f, R in outs[1:]:
        assert np.array_equal(f, outs[0][0]) and np.array_equal(R, outs[0][1])


def test_suspension_in_a_batch_equals_alone():
    ws = [small_suspension("f32", seed=s) for s in (1, 2)]
    ws.append(workloads.c1_small_fp64().with_(storage="f32"))
    print("[case] suspension batch", flush=True)
    alone = []
    for w in ws:
        with _lib.simulation_from_workload(w, storage="f32") as sim:
            sim.step(80)
            alone.append(sim.beads()[0])
    params = [_lib.params_from_mapping(w.params(), storage="f32") for w in ws]
    budget = sum(_lib.fpd_sim_footprint(p) for p in params) * 2
    with _lib.Batch(budget, len(ws), storage="f32") as b:
        ids = [b.add(p, w.beads(), 80) for p, w in zip(params, ws)]
        while b.run(32):
            pass
        for sid, R in zip(ids, alone):
            assert np.array_equal(b.beads(sid)[0], R)


def test_bead_count_must_divide_into_fibers():
    w = small_suspension("f64").with_(n_chains=5)
    with pytest.raises(_lib.FpdError) as e:
        _lib.Simulation(_lib.params_from_mapping(w.params(), storage="f64"))
    assert e.value.code == _lib.FPD_EINVAL


# ---------------------------------------------------------------- excluded volume ----

def touching_pair(storage, ev_k=0.05, cx=60.0, dy=2.6):
    """Two short fibers of beads of radius 1.5 laid across each other closer than 2a, in the
    +-U channel, with the excluded volume on."""
    centres = ((cx, 30.0, 0.2), (cx + 1.1, 30.0 + dy, -0.25))
    w = workloads.fiber_suspension(n_fibers=2, beads=4, nx=150, ny=60, radius=1.5,
                                   re_ps=2.0, kappa=0.5, u_wall=0.02, storage=storage)
    return w.with_(centres=centres, ev_k=ev_k)


@pytest.mark.parametrize("storage,tol_f,tol_r", [("f64", 1e-12, 1e-11), ("f32", 1e-5, 1e-4)])
def test_excluded_volume_matches_oracle(storage, tol_f, tol_r):
    w = touching_pair(storage)
    p = oracle.OracleParams.from_mapping(w.params())
    R0 = w.beads()
    F0 = oracle.bead_forces(p, R0)
    assert np.abs(F0 - oracle.bead_forces(oracle.OracleParams.from_mapping(
        w.with_(ev_k=0.0).params()), R0)).max() > 1e-3          # the repulsion acts
    print(f"[case] excluded volume {storage}", flush=True)
    st = oracle.make_state(p, 1, R0)
    oracle.run(st, 300)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        assert np.abs(sim.beads()[2] - F0).max() <= 1e-13 * np.abs(F0).max()  # read-back
        sim.step(300)
        sim.sync()
        f = sim.populations()
        R = sim.beads()[0]
        flags, _ = sim.health()
    assert flags == 0
    assert rel_err(f, st.f) <= tol_f
    assert np.max(np.abs(R - st.R)) <= tol_r


def test_excluded_volume_in_a_batch_and_across_the_periodic_boundary():
    # the pair straddles x = 0, so the minimum image decides which beads touch
    ws = [touching_pair("f32", cx=0.6), touching_pair("f32", ev_k=0.02)]
    print("[case] excluded volume batch", flush=True)
    alone = []
    for w in ws:
        with _lib.simulation_from_workload(w, storage="f32") as sim:
            sim.step(150)
            alone.append((sim.populations(), sim.beads()[0]))
    p = oracle.OracleParams.from_mapping(ws[0].params())
    st = oracle.make_state(p, 1, ws[0].beads())
    oracle.run(st, 150)
    assert np.max(np.abs(alone[0][1] - st.R)) <= 1e-4
    params = [_lib.params_from_mapping(w.params(), storage="f32") for w in ws]
    with _lib.Batch(4 * sum(_lib.fpd_sim_footprint(q) for q in params), 2, storage="f32") as b:
        ids = [b.add(q, w.beads(), 150) for q, w in zip(params, ws)]
        while b.run(64):
            pass
        for sid, (f, R) in zip(ids, alone):
            assert np.array_equal(b.populations(sid), f)
            assert np.array_equal(b.beads(sid)[0], R)
