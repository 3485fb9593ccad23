"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerances:
  * FPD_F64: populations and bead positions agree to round-off (1e-12 relative after 100
    steps, 1e-10 lu for beads after 1000 steps); differences come only from summation
    order and FMA contraction.
  * FPD_F32: populations within 1e-5 relative after 100 steps and bead positions within
    1e-4 lattice units after 1000 steps (the accuracy the FP32 path is held to).
"""
import ctypes
import math
import time

import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu


def orc_params(w):
    return oracle.OracleParams.from_mapping(w.params())


def gpu_sim(w, storage, **over):
    return _lib.simulation_from_workload(w, storage=storage, **over)


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def print_case(name, w, storage):
    print(f"[case] {name} {w.nx}x{w.ny} N={w.n_beads} storage={storage}", flush=True)


def small_fiber(nx, ny, n, seed, storage="f64", theta=None, l0=3.0, a=1.5):
    rng = np.random.default_rng(seed)
    th = rng.uniform(0, math.pi) if theta is None else theta
    reach = 0.5 * (n - 1) * l0 * abs(math.sin(th)) + a + 1.0 + 0.5
    cy = rng.uniform(reach, ny - reach) if ny > 2 * reach else ny / 2
    return workloads.Workload(
        name=f"rand{seed}", nx=nx, ny=ny, u_wall=0.02, nu_f=0.05, eta_ratio=20.0, xi=0.8,
        n_beads=n, radius=a, l0=l0, k_s=0.05 * l0 * l0, k_b=2e-3, theta0=th,
        cx=rng.uniform(0, nx), cy=cy, steps=0, storage=storage)


# ------------------------------------------------------------------ state and I/O ---

@pytest.mark.parametrize("storage,tol", [("f64", 1e-16), ("f32", 1e-7)])
def test_initial_populations_match_oracle(storage, tol):
    w = workloads.c1_small_fp64().with_(n_beads=0)
    print_case("init", w, storage)
    with gpu_sim(w, storage) as sim:
        f = sim.populations()
    ref = oracle.init(orc_params(w), 1)
    assert np.max(np.abs(f - ref)) <= tol


# f32 / f16dev / bf16dev store g = f - w with 24 / 11 / 8 significant bits; |g| < 6e-3 here
@pytest.mark.parametrize("storage,tol", [("f64", 0.0), ("f32", 6e-3 * 2.0 ** -24),
                                         ("f16dev", 6e-3 * 2.0 ** -11),
                                         ("bf16dev", 6e-3 * 2.0 ** -8)])
def test_write_read_roundtrip(storage, tol):
    w = workloads.c1_small_fp64().with_(nx=37, ny=11, n_beads=0)
    print_case("roundtrip", w, storage)
    f = oracle.init(orc_params(w), 1) + workloads.perturbation((9, 11, 37), 1e-3, seed=5)
    with gpu_sim(w, storage) as sim:
        sim.write_populations(f)
        g = sim.populations()
    assert np.max(np.abs(g - f)) <= tol


# -------------------------------------------------------------- lattice-only steps ---

@pytest.mark.parametrize("nx,ny", [(64, 32), (67, 13), (130, 7), (5, 3), (1, 4), (9, 1)])
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_lattice_steps_without_fiber(nx, ny, storage):
    w = workloads.c1_small_fp64().with_(nx=nx, ny=ny, n_beads=0, u_wall=0.03, nu_f=0.02)
    print_case("lattice", w, storage)
    p = orc_params(w)
    f0 = oracle.init(p, 1) + workloads.perturbation((9, ny, nx), 2e-3, seed=nx * 100 + ny)
    st = oracle.make_state(p, 1)
    st.f[:] = f0
    oracle.run(st, 100)
    with gpu_sim(w, storage) as sim:
        sim.write_populations(f0)
        sim.step(100)
        sim.sync()
        f = sim.populations()
    tol = 1e-12 if storage == "f64" else 1e-5
    assert rel_err(f, st.f) <= tol


# Two-byte storage moves populations as 32-bit words, two nodes per lane, with the
# neighbours' values passed between lanes: odd widths, widths that end inside a wave, and
# rows spanning several waves (130, 300) cover every edge case of that exchange.  The
# bound is the storage rounding (|g| < 2e-2 here; 11 / 8 significant bits, two roundings
# per step: the written state and each stored result) with a factor 2 of slack; a
# population taken from a wrong node would be off by the 5e-3 perturbation.
@pytest.mark.parametrize("nx,ny", [(64, 32), (67, 13), (130, 7), (300, 5), (5, 3), (1, 4),
                                   (9, 1), (2, 3)])
@pytest.mark.parametrize("storage,bits", [("f16dev", 11), ("bf16dev", 8)])
def test_two_byte_storage_steps_without_fiber(nx, ny, storage, bits):
    w = workloads.c1_small_fp64().with_(nx=nx, ny=ny, n_beads=0, u_wall=0.03, nu_f=0.02)
    print_case("lattice-2byte", w, storage)
    p = orc_params(w)
    f0 = oracle.init(p, 1) + workloads.perturbation((9, ny, nx), 5e-3, seed=nx * 7 + ny)
    gmax = float(np.abs(f0 - oracle.init(p, 1)).max()) + 0.03
    for steps in (1, 3):
        st = oracle.make_state(p, 1)
        st.f[:] = f0
        oracle.run(st, steps)
        with gpu_sim(w, storage) as sim:
            sim.write_populations(f0)
            sim.step(steps)
            sim.sync()
            f = sim.populations()
        tol = 2.0 * (steps + 1) * gmax * 2.0 ** -bits
        assert np.max(np.abs(f - st.f)) <= tol, (steps, np.max(np.abs(f - st.f)), tol)


# --------------------------------------------------------------- coupled fiber step ---

def run_both(w, storage, steps, record=None):
    p = orc_params(w)
    st = oracle.make_state(p, w.init_flow, w.beads())
    traj = oracle.run(st, steps, trajectory=record is not None)
    with gpu_sim(w, storage) as sim:
        sim.step(steps)
        sim.sync()
        f = sim.populations()
        R, V, F = sim.beads()
    return st, traj, f, R, V, F


def test_c1_fp64_populations_after_100_steps():
    w = workloads.c1_small_fp64()
    print_case("c1-100", w, "f64")
    st, _, f, R, V, F = run_both(w, "f64", 100)
    assert rel_err(f, st.f) <= 1e-12
    assert np.max(np.abs(R - st.R)) <= 1e-12
    assert np.max(np.abs(V - st.V)) <= 1e-14
    Fo = oracle.bead_forces(orc_params(w), st.R)
    assert np.max(np.abs(F - Fo)) <= 1e-9 * np.abs(Fo).max()


def test_c1_fp64_beads_after_1000_steps():
    w = workloads.c1_small_fp64()
    print_case("c1-1000", w, "f64")
    st, _, f, R, V, F = run_both(w, "f64", 1000)
    assert np.max(np.abs(R - st.R)) <= 1e-10
    assert rel_err(f, st.f) <= 1e-10


def test_c1_fp32_populations_after_100_steps():
    w = workloads.c1_small_fp64()
    print_case("c1-100", w, "f32")
    st, _, f, R, V, F = run_both(w, "f32", 100)
    assert rel_err(f, st.f) <= 1e-5


def test_c1_fp32_beads_after_1000_steps():
    w = workloads.c1_small_fp64()
    print_case("c1-1000", w, "f32")
    st, _, f, R, V, F = run_both(w, "f32", 1000)
    assert np.max(np.abs(R - st.R)) <= 1e-4


@pytest.mark.parametrize("nx,ny,n,seed", [(67, 29, 3, 1), (130, 40, 6, 2), (48, 23, 1, 3),
                                          (40, 31, 2, 4), (200, 45, 9, 5)])
@pytest.mark.parametrize("storage,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_ragged_lattices_with_fiber(nx, ny, n, seed, storage, tol):
    w = small_fiber(nx, ny, n, seed, storage)
    print_case(f"ragged-seed{seed}", w, storage)
    st, _, f, R, V, F = run_both(w, storage, 60)
    assert rel_err(f, st.f) <= tol
    assert np.max(np.abs(R - st.R)) <= (1e-11 if storage == "f64" else 1e-6)


@pytest.mark.parametrize("storage,tol,tol_r", [("f64", 1e-11, 1e-11), ("f32", 1e-5, 1e-6)])
def test_fiber_straddling_the_periodic_boundary(storage, tol, tol_r):
    """The fiber's support crosses x = 0: minimum images in FP64 and, for FP32 storage, the
    integer offsets plus FP32 fraction of the fiber tiles and the bead kernel."""
    w = small_fiber(96, 40, 5, 7, storage, theta=0.2).with_(cx=1.0)
    print_case("wrap", w, storage)
    st, _, f, R, V, F = run_both(w, storage, 80)
    assert rel_err(f, st.f) <= tol
    assert np.max(np.abs(R - st.R)) <= tol_r
    assert st.R[:, 0].min() < 1.0 and (st.R[:, 0].min() < 0 or st.R[:, 0].max() > 95)


def test_fields_match_oracle():
    w = workloads.c1_small_fp64()
    print_case("fields", w, "f64")
    p = orc_params(w)
    st = oracle.make_state(p, 1, w.beads())
    oracle.run(st, 50)
    rho_o, ux_o, uy_o, eta_o = oracle.macro(p, st.f, st.R)
    with gpu_sim(w, "f64") as sim:
        sim.step(50)
        rho, ux, uy, eta = sim.fields()
    assert np.max(np.abs(rho - rho_o)) <= 1e-13
    assert np.max(np.abs(ux - ux_o)) <= 1e-13
    assert np.max(np.abs(uy - uy_o)) <= 1e-13
    assert np.max(np.abs(eta - eta_o) / eta_o) <= 1e-12


# ------------------------------------------------------------ launch and replay paths ---

LAUNCHES = [
    dict(block_x=64, block_y=4, rows_per_thread=1, xcd_remap=1),
    dict(block_x=128, block_y=2, rows_per_thread=2, xcd_remap=2),
    dict(block_x=256, block_y=1, rows_per_thread=4, xcd_remap=1),
    dict(block_x=64, block_y=1, rows_per_thread=2, xcd_remap=2),
    dict(block_x=256, block_y=1, rows_per_thread=1, xcd_remap=2),
    dict(block_x=128, block_y=2, rows_per_thread=1, xcd_remap=2),
]


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_launch_shapes_and_graph_replay_are_bitwise_identical(storage):
    w = small_fiber(150, 37, 6, 11, storage)
    print_case("launch-shapes", w, storage)
    outs = []
    for i, cfg in enumerate(LAUNCHES):
        for flags in (0, _lib.FPD_FLAG_NO_GRAPH):
            with gpu_sim(w, storage, flags=flags) as sim:
                sim.set_launch(dict(cfg, graph_chunk=8))
                sim.step(3)        # direct launches
                sim.step(16)       # two graph replays unless NO_GRAPH
                sim.step(5)
                sim.sync()
                outs.append((sim.populations(), sim.beads()[0]))
    for f, R in outs[1:]:
        assert np.array_equal(f, outs[0][0])
        assert np.array_equal(R, outs[0][1])


def test_timed_path_matches_untimed():
    w = workloads.c1_small_fp64()
    print_case("timed", w, "f32")
    with gpu_sim(w, "f32", flags=_lib.FPD_FLAG_TIME_KERNELS) as a, gpu_sim(w, "f32") as b:
        a.sync()
        t0 = time.perf_counter()
        a.step(40)
        a.sync()
        wall_ms = (time.perf_counter() - t0) * 1e3
        b.step(40)
        assert np.array_equal(a.populations(), b.populations())
        ms_l, n_l, ms_b, n_b = a.kernel_times()
        assert n_l == 40 and n_b == 40 and ms_l > 0 and ms_b > 0
        # the durations are those of the dispatches, which run one after another on the
        # simulation's stream: together they fit in the host's wall time of those steps
        assert ms_l + ms_b <= wall_ms, (ms_l, ms_b, wall_ms)


def test_repeat_runs_are_deterministic():
    w = small_fiber(120, 44, 8, 13, "f64")
    print_case("determinism", w, "f64")
    res = []
    for _ in range(2):
        with gpu_sim(w, "f64") as sim:
            sim.step(70)
            res.append((sim.populations(), sim.beads()))
    assert np.array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("first", [100, 101])
def test_checkpoint_resume_is_bitwise(tmp_path, first):
    w = workloads.c1_small_fp64()
    print_case(f"checkpoint-{first}", w, "f32")
    path = str(tmp_path / "c1.fpd")
    with gpu_sim(w, "f32") as a:
        a.step(200)
        fa, Ra = a.populations(), a.beads()[0]
    with gpu_sim(w, "f32") as b:
        b.step(first)
        b.save(path)
    with gpu_sim(w, "f32") as c:
        c.load(path)
        assert c.steps == first
        c.step(200 - first)
        assert np.array_equal(c.populations(), fa)
        assert np.array_equal(c.beads()[0], Ra)


@pytest.mark.parametrize("over", [dict(g_body=(1e-7, 0.0)), dict(flags=_lib.FPD_FLAG_CLAMP_PHI),
                                  dict(k_b=0.5), dict(n_chains=5)])
def test_checkpoint_of_another_problem_is_refused(tmp_path, over):
    w = workloads.c1_small_fp64()
    print_case(f"checkpoint-mismatch-{sorted(over)}", w, "f32")
    path = str(tmp_path / "c1.fpd")
    with gpu_sim(w, "f32") as a:
        a.step(4)
        a.save(path)
    with gpu_sim(w, "f32", **over) as b:
        with pytest.raises(_lib.FpdError) as err:
            b.load(path)
        assert err.value.code == _lib.FPD_EINVAL and "does not match" in str(err.value)
        assert b.steps == 0


def hip_runtime():
    """The HIP runtime the library links (already loaded with it), for raw allocations."""
    _lib.lib()
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
    hip.hipFree.argtypes = [ctypes.c_void_p]
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    return hip


def test_caller_owned_buffers():
    """fpd_create_with_buffers: the state lives in the caller's device memory and the steps
    are bitwise those of library-owned buffers; short or misaligned buffers are refused."""
    w = workloads.c1_small_fp64()
    print_case("caller-buffers", w, "f32")
    p = _lib.params_from_mapping(w.params(), storage="f32")
    n = _lib.fpd_population_bytes(p)
    hip = hip_runtime()
    ptrs = []
    try:
        for _ in range(2):
            ptr = ctypes.c_void_p()
            assert hip.hipMalloc(ctypes.byref(ptr), n) == 0
            ptrs.append(ptr.value)

        def snapshot():
            out = np.empty(n, np.uint8)
            assert hip.hipMemcpy(out.ctypes.data, ptrs[0], n, 2) == 0  # device to host
            return out

        with _lib.Simulation(p, buffers=(ptrs[0], ptrs[1], n)) as a, gpu_sim(w, "f32") as b:
            a.init_fiber(w.beads())
            a.step(30)
            b.step(30)
            assert np.array_equal(a.populations(), b.populations())
            assert np.array_equal(a.beads()[0], b.beads()[0])
            a.sync()
            before = snapshot()
            a.step(2)  # buffer 0 is written again every second step
            a.sync()
            assert not np.array_equal(snapshot(), before)
        with pytest.raises(_lib.FpdError) as err:
            _lib.Simulation(p, buffers=(ptrs[0], ptrs[1], n - 64))
        assert err.value.code == _lib.FPD_EINVAL
        with pytest.raises(_lib.FpdError) as err:  # not 16-byte aligned
            _lib.Simulation(p, buffers=(ptrs[0] + 8, ptrs[1], n - 8))
        assert err.value.code == _lib.FPD_EINVAL
    finally:
        for ptr in ptrs:
            hip.hipFree(ptr)


def test_zero_steps_is_a_no_op():
    w = workloads.c1_small_fp64()
    with gpu_sim(w, "f64") as sim:
        f0 = sim.populations()
        sim.step(0)
        assert np.array_equal(sim.populations(), f0)
        assert sim.steps == 0


# ------------------------------------------------------------------- health ---------

def test_nan_populations_raise_unstable_and_stay_local():
    w = workloads.c1_small_fp64()
    print_case("health", w, "f32")
    with gpu_sim(w, "f32") as bad, gpu_sim(w, "f32") as good:
        f = bad.populations()
        f[:, 14:18, 30:34] = np.nan
        bad.write_populations(f)
        bad.step(5)
        good.step(5)
        with pytest.raises(_lib.FpdError) as e:
            bad.sync()
        assert e.value.code == _lib.FPD_EUNSTABLE
        good.sync()
        flags, strain = bad.health()
        assert flags & _lib.FPD_HEALTH_NAN


def test_invalid_fiber_is_rejected():
    w = workloads.c1_small_fp64()
    with gpu_sim(w.with_(n_beads=5), "f32") as sim:
        R = w.beads().copy()
        R[0, 1] = 0.5          # inside the wall layer
        with pytest.raises(_lib.FpdError) as e:
            sim.init_fiber(R)
        assert e.value.code == _lib.FPD_EINVAL
