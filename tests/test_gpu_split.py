"""Split steps against whole steps.  A split step runs the lattice update as two kernels:
the tiles away from the fiber on a second stream, overlapping the bead kernel of the step
before, and the tiles of the partition around the fiber after it.  Every tile runs the
code of the one-kernel step, so populations and beads must be the same bits, for every
storage format, with and without graph replay, across the periodic edges, with a body
force, and for launch shapes whose tiles do not divide the lattice."""
import math

import numpy as np
import pytest

import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu


def fiber(nx, ny, storage, cx, cy, theta, boundary=0, **over):
    kw = dict(name="split", nx=nx, ny=ny, u_wall=0.02, nu_f=0.05, eta_ratio=20.0, xi=0.8,
              n_beads=10, radius=1.5, l0=3.0, k_s=0.45, k_b=2e-3, theta0=theta, cx=cx,
              cy=cy, steps=0, storage=storage, boundary=boundary)
    if boundary == 1:
        kw.update(u_wall=0.0, init_flow=0, f_ext=(2e-4, 1e-4))
    kw.update(over)
    return workloads.Workload(**kw)


def run(w, flags, launch=None, chunk=8):
    with _lib.simulation_from_workload(w, storage=w.storage, flags=flags) as sim:
        if launch:
            sim.set_launch(dict(launch, graph_chunk=chunk))
        else:
            sim.set_launch(dict(graph_chunk=chunk))
        split = sim.split_active()
        sim.step(3)        # a whole first step, then direct split steps
        sim.step(2 * chunk)  # graph replays unless FPD_FLAG_NO_GRAPH
        sim.step(5)
        sim.sync()
        return split, sim.populations(), sim.beads()
    

def compare(w, launch=None):
    print(f"[case] split {w.nx}x{w.ny} {w.storage} boundary={w.boundary} launch={launch}",
          flush=True)
    on, f0, b0 = run(w, _lib.FPD_FLAG_NO_SPLIT, launch)
    assert not on
    for flags in (0, _lib.FPD_FLAG_NO_GRAPH):
        on, f, b = run(w, flags, launch)
        assert on, "the split path was not taken"
        assert np.array_equal(f, f0)
        for x, y in zip(b, b0):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_split_steps_are_bitwise_whole_steps(storage):
    compare(fiber(1024, 384, storage, cx=400.0, cy=190.0, theta=0.7))


@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev"])
def test_split_across_the_periodic_x_edge(storage):
    """The partition wraps around x = 0 (its tiles run from the last, narrow one on)."""
    compare(fiber(1000, 384, storage, cx=2.0, cy=150.0, theta=0.3))


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_split_in_a_periodic_box_corner(storage):
    """No walls: the partition wraps in x and y at once; a driven fiber."""
    compare(fiber(768, 512, storage, cx=1.0, cy=2.0, theta=0.9, boundary=1))


def test_split_with_a_body_force():
    """Fluid tiles take the forced collision when a body force acts everywhere."""
    compare(fiber(1024, 384, "f32", cx=512.0, cy=192.0, theta=2.0, g_body=(1e-6, 0.0)))


@pytest.mark.parametrize("launch", [
    dict(block_x=128, block_y=2, rows_per_thread=2, xcd_remap=1),
    dict(block_x=64, block_y=4, rows_per_thread=1, xcd_remap=2),
    dict(block_x=256, block_y=1, rows_per_thread=4, xcd_remap=1),
])
@pytest.mark.parametrize("storage", ["f32", "bf16dev"])
def test_split_with_other_launch_shapes(storage, launch):
    compare(fiber(1000, 390, storage, cx=990.0, cy=200.0, theta=2.4), launch)


@pytest.mark.parametrize("storage", ["f64", "f16dev"])
def test_timed_split_steps_match_untimed(storage):
    """FPD_FLAG_TIME_KERNELS keeps split steps (direct launches, each kernel stamped): the
    same bits as graph-replayed split steps; the first step after the fiber runs whole and
    untimed; a lattice pass spans its fluid and fiber kernels."""
    w = fiber(1024, 384, storage, cx=400.0, cy=190.0, theta=0.7)
    print(f"[case] timed split {storage}", flush=True)
    with _lib.simulation_from_workload(w, storage=storage,
                                       flags=_lib.FPD_FLAG_TIME_KERNELS) as a, \
            _lib.simulation_from_workload(w, storage=storage) as b:
        assert a.split_active()
        a.step(31)
        b.set_launch(dict(graph_chunk=10))
        b.step(31)
        a.sync()
        b.sync()
        assert np.array_equal(a.populations(), b.populations())
        assert np.array_equal(a.beads()[0], b.beads()[0])
        ms_l, n_l, ms_b, n_b = a.kernel_times()
        assert n_l == 30 and n_b == 30 and ms_l > 0 and ms_b > 0


def test_split_with_the_fiber_ends_recorder():
    """The recorder's kernel runs on the fiber stream ahead of each fiber kernel, beside
    the fluid kernel: the same records and state as with whole steps."""
    w = fiber(1024, 384, "f32", cx=400.0, cy=190.0, theta=0.7)
    print("[case] split with recorder", flush=True)
    out = []
    for flags in (_lib.FPD_FLAG_NO_SPLIT, 0):
        with _lib.simulation_from_workload(w, storage="f32", flags=flags) as sim:
            sim.set_launch(dict(graph_chunk=8))
            sim.record_start(every=3, capacity=64)
            sim.step(40)
            sim.sync()
            out.append((sim.split_active(), sim.record(), sim.populations()))
    assert not out[0][0] and out[1][0]
    assert out[0][1].shape[0] >= 13
    assert np.array_equal(out[0][1], out[1][1])
    assert np.array_equal(out[0][2], out[1][2])


def test_split_not_taken_where_it_cannot_pay():
    """A partition of more than a quarter of the tiles (a small lattice) or a fixed
    profile: whole steps."""
    w = fiber(96, 40, "f32", cx=48.0, cy=20.0, theta=0.2, n_beads=5)
    with _lib.simulation_from_workload(w, storage="f32") as sim:
        assert not sim.split_active()
    w = fiber(1024, 384, "f32", cx=400.0, cy=190.0, theta=0.7)
    with _lib.simulation_from_workload(w, storage="f32") as sim:
        assert sim.split_active()
        sim.set_flags(_lib.FPD_FLAG_NO_SPLIT)
        assert not sim.split_active()
        sim.set_flags(_lib.FPD_FLAG_TIME_KERNELS)  # timed steps stay split
        assert sim.split_active()
        sim.set_flags(0)
        assert sim.split_active()
        sim.set_static_phi(np.zeros(w.ny))
        assert not sim.split_active()


def test_capture_right_after_the_fiber():
    """fpd_capture right after fpd_init_fiber captures the graph of the steps after the
    whole first one; the run matches one without the capture."""
    w = fiber(1024, 384, "f32", cx=400.0, cy=190.0, theta=0.7)
    print("[case] capture after init", flush=True)
    with _lib.simulation_from_workload(w, storage="f32") as a, \
            _lib.simulation_from_workload(w, storage="f32", flags=_lib.FPD_FLAG_NO_SPLIT) as b:
        a.set_launch(dict(graph_chunk=8))
        a.capture(17)
        a.step(17)
        b.step(17)
        a.sync()
        b.sync()
        assert np.array_equal(a.populations(), b.populations())
        assert np.array_equal(a.beads()[0], b.beads()[0])


def test_split_after_save_and_load(tmp_path):
    """After fpd_load the first step runs whole (the stored partition is not trusted) and
    the run continues as if uninterrupted."""
    w = fiber(1024, 384, "f32", cx=400.0, cy=190.0, theta=0.7)
    path = str(tmp_path / "state.fpd")
    with _lib.simulation_from_workload(w, storage="f32") as a:
        a.step(7)
        a.save(path)
        a.step(9)
        a.sync()
        f_ref, R_ref = a.populations(), a.beads()[0]
    with _lib.simulation_from_workload(w, storage="f32") as b:
        b.load(path)
        b.step(9)
        b.sync()
        assert np.array_equal(b.populations(), f_ref)
        assert np.array_equal(b.beads()[0], R_ref)
