"""GPU parity at the full sizes of the throughput runs, in the launch configuration that the
benchmark times (the default launch shape, steps replayed from a captured graph).

  * 8192 x 2048 channel with the 40-bead fiber (16.8M nodes), FP64 and FP32 storage: every
    population and every bead after two coupled steps against the FP64 oracle on the same
    lattice (the oracle needs about 2.5 s per step here); FP16 / BF16 deviation storage
    against the same oracle state within the storage rounding;
  * 1024 x 256 channel with the 20-bead fiber: every population after 100 steps;
  * properties that hold at any size, over the benchmark's 2000 steps at 8192 x 2048: total
    mass is conserved (tangential walls, mass-preserving collision), and the fiber centred
    in the +-U channel stays point-symmetric about the centre (rotation by 180 degrees maps
    the problem onto itself).

Tolerances as for the small cases: FP64 1e-12 relative on populations, FP32 1e-5.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
# two-byte deviation storage: significant bits of binary16 / bfloat16
BITS = {"f16dev": 11, "bf16dev": 8}


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


@pytest.fixture(scope="module")
def c3_oracle():
    w = workloads.c3_large("f64")
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, w.init_flow, w.beads())
    oracle.run(st, 2)
    return st


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_c3_full_size_two_steps_match_oracle(c3_oracle, storage):
    w = workloads.c3_large(storage)
    print(f"[case] c3 full size {w.nx}x{w.ny} N={w.n_beads} storage={storage}", flush=True)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.set_launch(dict(graph_chunk=2))    # the two steps run as one graph replay
        sim.step(2)
        sim.sync()
        f = sim.populations()
        R, V, _ = sim.beads()
    assert rel_err(f, c3_oracle.f) <= TOL[storage]
    tol_r = 1e-12 if storage == "f64" else 1e-6
    assert np.max(np.abs(R - c3_oracle.R)) <= tol_r
    assert np.max(np.abs(V - c3_oracle.V)) <= tol_r


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_c3_full_size_two_steps_two_byte_storage(c3_oracle, storage):
    """The two-byte formats at full size in the benchmark's launch shape: every population
    within the storage rounding of the oracle's, as for the small lattices (11 / 8
    significant bits, two roundings per step: the written state and each stored result,
    a factor 2 of slack), and the beads within the rounding that reaches Eq. (5): a
    momentum component sums six populations, each off by at most that bound."""
    w = workloads.c3_large(storage)
    print(f"[case] c3 full size {w.nx}x{w.ny} N={w.n_beads} storage={storage}", flush=True)
    p = oracle.OracleParams.from_mapping(w.params())
    steps = 2
    # largest deviation |f - w| of the state (the rest state is f = w), with 50 % margin
    gmax = 1.5 * float(np.abs(c3_oracle.f - oracle.init(p, 0)).max())
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.set_launch(dict(graph_chunk=2))
        sim.step(steps)
        sim.sync()
        f = sim.populations()
        R, V, _ = sim.beads()
    tol = 2.0 * (steps + 1) * gmax * 2.0 ** -BITS[storage]
    err = float(np.max(np.abs(f - c3_oracle.f)))
    print(f"[c3 {storage}] population err {err:.3e} (bound {tol:.3e})", flush=True)
    assert err <= tol
    tol_v = 6.0 * tol
    assert np.max(np.abs(V - c3_oracle.V)) <= tol_v
    assert np.max(np.abs(R - c3_oracle.R)) <= steps * tol_v


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_c2_full_size_matches_oracle(storage):
    w = workloads.c2_medium_fp32().with_(storage=storage)
    print(f"[case] c2 full size {w.nx}x{w.ny} N={w.n_beads} storage={storage}", flush=True)
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, w.init_flow, w.beads())
    oracle.run(st, 100)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.step(100)
        sim.sync()
        f = sim.populations()
        R, _, _ = sim.beads()
    assert rel_err(f, st.f) <= TOL[storage]
    assert np.max(np.abs(R - st.R)) <= (1e-11 if storage == "f64" else 1e-5)


@pytest.mark.parametrize("storage,tol_mass,tol_sym", [("f64", 1e-12, 1e-9),
                                                      ("f32", 1e-6, 2e-3)])
def test_c3_bench_run_conserves_mass_and_point_symmetry(storage, tol_mass, tol_sym):
    w = workloads.c3_large(storage)
    print(f"[case] c3 {w.steps} steps properties storage={storage}", flush=True)
    c = np.array([w.cx, w.cy])
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.step(w.steps)
        sim.sync()
        flags, _ = sim.health()
        rho, _, _, _ = sim.fields()
        R, _, _ = sim.beads()
    assert flags == 0
    assert abs(float(np.sum(rho - 1.0))) / rho.size <= tol_mass
    assert np.abs(R + R[::-1] - 2 * c).max() <= tol_sym
    # the fiber has moved (it turns clockwise in this shear)
    R0 = w.beads()
    d0, d1 = R0[-1] - R0[0], R[-1] - R[0]
    assert np.arctan2(d1[1], d1[0]) < np.arctan2(d0[1], d0[0])


def test_buffer_beyond_2_31_values():
    """Row offsets are 64-bit: a 16384 x 16384 FP16 lattice holds 2.4e9 values per buffer
    (rows past 2^31 / (9 x 16384) = 14563 start beyond 2^31).  The flow is uniform in x (a
    linear Couette start without a fiber), so after two steps every column equals the one
    column of a 64 x 16384 lattice, bitwise, up to the last row."""
    ny = 16384
    base = workloads.c1_small_fp64().with_(n_beads=0, ny=ny, u_wall=0.05, nu_f=0.05)
    print(f"[case] 16384x{ny} f16dev, 2 steps", flush=True)
    with _lib.simulation_from_workload(base.with_(nx=64), storage="f16dev") as sim:
        sim.step(2)
        sim.sync()
        _, ref, _, _ = sim.fields()
    big = base.with_(nx=16384)
    assert 9 * big.nx * (ny - 1) > 2 ** 31
    p = _lib.params_from_mapping(big.params(), storage="f16dev")
    with _lib.Simulation(p) as sim:
        sim.step(2)
        sim.sync()
        ux = np.empty((ny, big.nx))
        _lib.check(_lib.lib().fpd_read_fields(sim.h, None, _lib._ptr(ux), None, None))
    assert np.array_equal(ux, np.broadcast_to(ref[:, :1], ux.shape))
    assert abs(ux[-1, 0]) > 0.9 * 0.05                     # the top row moved with the wall
