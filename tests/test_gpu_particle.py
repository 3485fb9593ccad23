"""GPU parity for the driven-particle benchmark of Sec. III.B: the periodic box (no walls),
the external force on the beads with the balancing body force, and the on-device
diagnostics (eps_v of Eq. 15, drag of Eq. 17 in diffuse-interface form) against the
oracle, through the C ABI.

Tolerances as for the channel runs: FP64 populations 1e-12 relative, FP32 1e-5; two-byte
storage within its rounding.  The diagnostics on one FP64 state agree to 1e-9 relative
(FP64 sums in another order; eps_v is a difference of nearly equal velocities and gets
1e-7).
"""
import math

import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def orc_params(w):
    return oracle.OracleParams.from_mapping(w.params())


@pytest.mark.parametrize("nx,ny", [(48, 48), (67, 13), (130, 7), (5, 3), (1, 4), (9, 1)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_periodic_box_lattice_steps(nx, ny, storage):
    w = workloads.driven_particle(storage=storage).with_(nx=nx, ny=ny, n_beads=0,
                                                          g_body=(2e-6, -1e-6))
    print(f"[case] periodic lattice {nx}x{ny} {storage}", flush=True)
    p = orc_params(w)
    f0 = oracle.init(p, 0) + workloads.perturbation((9, ny, nx), 5e-3, seed=nx * 31 + ny)
    steps = 3 if storage in ("f16dev", "bf16dev") else 50
    st = oracle.make_state(p, 0)
    st.f[:] = f0
    oracle.run(st, steps)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.write_populations(f0)
        sim.step(steps)
        sim.sync()
        f = sim.populations()
    if storage == "f64":
        assert rel_err(f, st.f) <= 1e-12
    elif storage == "f32":
        assert rel_err(f, st.f) <= 1e-5
    else:
        bits = 11 if storage == "f16dev" else 8
        gmax = float(np.abs(f0 - oracle.init(p, 0)).max()) + 0.02
        assert np.max(np.abs(f - st.f)) <= 2.0 * (steps + 1) * gmax * 2.0 ** -bits


@pytest.mark.parametrize("storage,steps,tol_f,tol_r", [("f64", 300, 1e-12, 1e-12),
                                                       ("f32", 300, 1e-5, 1e-6)])
def test_driven_particle_matches_oracle(storage, steps, tol_f, tol_r):
    w = workloads.driven_particle(n=48, radius=3.0, storage=storage, force=2e-4)
    print(f"[case] driven particle {storage} {steps}", flush=True)
    st = oracle.make_state(orc_params(w), 0, w.beads())
    oracle.run(st, steps)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.step(steps)
        sim.sync()
        f = sim.populations()
        R, V, F = sim.beads()
    assert rel_err(f, st.f) <= tol_f
    assert np.max(np.abs(R - st.R)) <= tol_r
    assert np.max(np.abs(V - st.V)) <= tol_r * 1e-2
    assert np.max(np.abs(F - [2e-4, 0.0])) <= 1e-18     # F = F0 (one bead, no bonds)


def check_stats(g, o):
    scale_v = math.hypot(o["V0x"], o["V0y"]) + 1e-300
    scale_f = max(abs(o["Fvisc_x"]), abs(o["Fvisc_y"]), abs(o["Fpres_x"]), abs(o["Fpres_y"]))
    assert g["A"] == pytest.approx(o["A"], rel=1e-12)
    assert abs(g["V0x"] - o["V0x"]) <= 1e-9 * scale_v
    assert abs(g["V0y"] - o["V0y"]) <= 1e-9 * scale_v
    assert g["eps_v"] == pytest.approx(o["eps_v"], rel=1e-7, abs=1e-30)
    for k in ("Fvisc_x", "Fvisc_y", "Fpres_x", "Fpres_y"):
        assert abs(g[k] - o[k]) <= 1e-9 * scale_f, k


@pytest.mark.parametrize("n,radius,xi", [(48, 3.0, 1.0), (96, 4.0, 1.0)])
def test_particle_stats_match_oracle(n, radius, xi):
    # n = 48: the FP64 support (a + 20 xi) wraps the whole box; n = 96: a box inside
    w = workloads.driven_particle(n=n, radius=radius, xi=xi, storage="f64", force=2e-4)
    print(f"[case] particle stats {n}", flush=True)
    p = orc_params(w)
    st = oracle.make_state(p, 0, w.beads())
    oracle.run(st, 200)
    with _lib.simulation_from_workload(w, storage="f64") as sim:
        sim.step(200)
        g = sim.particle_stats(0)
        f = sim.populations()
        R = sim.beads()[0]
    assert rel_err(f, st.f) <= 1e-12
    # the oracle's diagnostics on the GPU's own state and on its own state
    check_stats(g, oracle.particle_stats(p, f, R))
    check_stats(g, oracle.particle_stats(p, st.f, st.R))
    assert g["Fvisc_x"] < 0 and g["V0x"] > 0          # drag opposes the motion


def test_particle_stats_in_a_channel_and_near_a_wall():
    w = workloads.c1_small_fp64().with_(nx=96, ny=72, n_beads=1, radius=4.0, u_wall=0.01,
                                        cx=40.3, cy=36.2, k_s=0.0, k_b=0.0)
    print("[case] particle stats channel", flush=True)
    p = orc_params(w)
    st = oracle.make_state(p, w.init_flow, w.beads())
    oracle.run(st, 50)
    with _lib.simulation_from_workload(w, storage="f64") as sim:
        sim.step(50)
        g = sim.particle_stats(0)
        f = sim.populations()
        R = sim.beads()[0]
    check_stats(g, oracle.particle_stats(p, f, R))
    near = w.with_(ny=40, cy=20.0)
    with _lib.simulation_from_workload(near, storage="f64") as sim:
        with pytest.raises(_lib.FpdError) as e:
            sim.particle_stats(0)
        assert e.value.code == _lib.FPD_EINVAL
        with pytest.raises(_lib.FpdError):
            sim.particle_stats(1)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_fiber_crossing_the_periodic_y_boundary(storage, tol):
    w = workloads.Workload(
        name="wrap_y", nx=40, ny=36, u_wall=0.0, nu_f=0.08, eta_ratio=20.0, xi=0.8,
        n_beads=4, radius=1.5, l0=3.0, k_s=0.05 * 9.0, k_b=2e-3, theta0=math.pi / 2 - 0.3,
        cx=17.3, cy=0.4, steps=0, storage=storage, init_flow=0, boundary=1,
        f_ext=(1e-4, 2e-4), g_body=(-4e-4 / 1440, -8e-4 / 1440))
    print(f"[case] fiber across y {storage}", flush=True)
    st = oracle.make_state(orc_params(w), 0, w.beads())
    oracle.run(st, 150)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.step(150)
        sim.sync()
        f = sim.populations()
        R = sim.beads()[0]
    assert rel_err(f, st.f) <= tol
    assert np.max(np.abs(R - st.R)) <= (1e-11 if storage == "f64" else 1e-5)
    assert st.R[:, 1].min() < 0 < st.R[:, 1].max()    # the fiber does straddle y = 0


def test_periodic_parameters_are_validated():
    w = workloads.driven_particle()
    for bad in (dict(u_wall=0.01), dict(init_flow=1), dict(boundary=2)):
        p = _lib.params_from_mapping(w.with_(**bad).params(), storage="f64")
        with pytest.raises(_lib.FpdError) as e:
            _lib.Simulation(p)
        assert e.value.code == _lib.FPD_EINVAL


def test_driven_particle_batch_equals_alone():
    ws = [workloads.driven_particle(n=40 + 8 * i, radius=3.0, storage="f32",
                                    force=1e-4 * (i + 1)) for i in range(3)]
    ws.append(workloads.c1_small_fp64().with_(storage="f32"))
    print("[case] batch with periodic boxes", flush=True)
    alone = []
    for w in ws:
        with _lib.simulation_from_workload(w, storage="f32") as sim:
            sim.step(90)
            alone.append((sim.populations(), sim.beads()[0]))
    params = [_lib.params_from_mapping(w.params(), storage="f32") for w in ws]
    budget = sum(_lib.fpd_sim_footprint(p) for p in params) * 2
    with _lib.Batch(budget, len(ws), storage="f32") as b:
        ids = [b.add(p, w.beads(), 90) for p, w in zip(params, ws)]
        while b.run(64):
            pass
        for sid, (f, R) in zip(ids, alone):
            assert np.array_equal(b.populations(sid), f)
            assert np.array_equal(b.beads(sid)[0], R)


def test_batch_particle_stats_equal_the_single_simulation():
    w = workloads.driven_particle(n=64, radius=4.0, storage="f64", force=3e-4)
    print("[case] batch particle stats", flush=True)
    with _lib.simulation_from_workload(w, storage="f64") as sim:
        sim.step(120)
        alone = sim.particle_stats(0)
    p = _lib.params_from_mapping(w.params(), storage="f64")
    with _lib.Batch(4 * _lib.fpd_sim_footprint(p), 2, storage="f64") as b:
        sid = b.add(p, w.beads(), 120)
        while b.run(64):
            pass
        assert b.particle_stats(sid) == alone
