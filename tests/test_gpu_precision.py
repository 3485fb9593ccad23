"""Reduced-precision population storage against the FP64 oracle (C1 workload).

FP16 / BF16 deviation storage (g = f - w kept in 11 / 8 significant bits, collision in
FP32) has no a-priori error bound; the errors are measured here and held to the stated
levels: the velocity field relative to the wall speed U, bead positions in lattice
units, after 1000 steps of the 64x32 channel with the 5-bead fiber.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu

# storage: (max |u - u_oracle| / U, max |R - R_oracle| in lu) after 1000 steps.  Measured on
# MI355X: f32 1.7e-5 U / 9.6e-6 lu, f16dev 1.0e-3 U / 1.8e-4 lu, bf16dev 1.2e-2 U /
# 1.6e-3 lu; over six starts shifted by 0 .. 5e-7 lu (an earlier build) f16dev
# 0.9-1.2e-3 U / 0.9-3.7e-4 lu and bf16dev 1.0-1.5e-2 U / 1.4-2.5e-3 lu (the two-byte
# rounding makes the bead error of one start vary by an order of magnitude).
BOUNDS = {"f32": (5e-5, 1e-4), "f16dev": (5e-3, 2e-3), "bf16dev": (5e-2, 5e-3)}


@pytest.fixture(scope="module")
def reference():
    w = workloads.c1_small_fp64()
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, 1, w.beads())
    oracle.run(st, 1000)
    rho, ux, uy, eta = oracle.macro(p, st.f, st.R)
    return w, st, ux, uy


@pytest.mark.parametrize("storage", ["f32", "f16dev", "bf16dev"])
def test_reduced_storage_error_against_oracle(reference, storage):
    w, st, ux_o, uy_o = reference
    print(f"[case] precision {storage}", flush=True)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.step(1000)
        sim.sync()
        rho, ux, uy, eta = sim.fields()
        R = sim.beads()[0]
    eu = max(np.abs(ux - ux_o).max(), np.abs(uy - uy_o).max()) / w.u_wall
    er = float(np.abs(R - st.R).max())
    print(f"[precision] {storage}: velocity err {eu:.3e} U, bead err {er:.3e} lu", flush=True)
    bu, br = BOUNDS[storage]
    assert eu <= bu and er <= br


# A simulation shaped like the served sweep (C5: N_y = 64, the smallest sweep size, N_x = 128,
# parameters drawn from the sweep's distributions, seed 1: 6 beads, C = 0.49, Re_ps = 9.8,
# K = 7.0, U = 0.042) over the served 20k steps (gamma t = 26), against the oracle at 1k,
# 5k and 20k steps.  Up to 5k steps the errors are stable and held to the measured levels
# with margin.  At 20k steps the fiber is flipping, and the two-byte storages' bead error
# is set by the phase of the flip: over starts shifted by 0 .. 5e-7 lu it spans
# 1.3 - 8.7 lu (FP16) and 0.13 - 1.9 lu (BF16), and 0.17 - 12 lu in a build that differs
# only in rounding, so there it is held as a distribution over six such starts (each against the FP64 path from the same start, which the oracle pins at
# the first one) by its median and its maximum.
SWEEP_BOUNDS = {"f64": (1e-10, 1e-10), "f32": (2e-4, 1e-3), "f16dev": (2e-2, 0.15),
                "bf16dev": (6e-2, 1.0)}
# two-byte storages at 20k steps: (median, max) over the six starts of the velocity error
# in U and of the bead error in lu (the fiber is 31 lu long)
FLIP_BOUNDS = {"f16dev": ((0.1, 0.25), (6.0, 16.0)), "bf16dev": ((0.1, 0.25), (6.0, 16.0))}


def _sweep_errors(w, storage, R0, ref):
    """Velocity (in U) and bead (lu) errors of `storage` from start R0 at each mark of ref
    (mark -> (ux, uy, R))."""
    p = _lib.params_from_mapping(w.params(), storage=storage)
    out, done = {}, 0
    with _lib.Simulation(p) as sim:
        sim.init_fiber(R0)
        for m in sorted(ref):
            sim.step(m - done)
            done = m
            sim.sync()
            _, ux, uy, _ = sim.fields()
            ux_o, uy_o, R_o = ref[m]
            eu = max(np.abs(ux - ux_o).max(), np.abs(uy - uy_o).max()) / w.u_wall
            out[m] = (eu, float(np.abs(sim.beads()[0] - R_o).max()), (ux, uy, sim.beads()[0]))
    return out


@pytest.mark.slow
def test_sweep_simulation_error_over_the_served_steps():
    w = workloads.sweep_sim_at_height(64, seed=1, storage="f64")
    print(f"[case] sweep-shaped {w.nx}x{w.ny} N={w.n_beads} 20k steps", flush=True)
    p = oracle.OracleParams.from_mapping(w.params())
    st = oracle.make_state(p, 1, w.beads())
    marks = (1000, 5000, 20000)
    ref, done = {}, 0
    for m in marks:
        oracle.run(st, m - done)
        done = m
        _, ux, uy, _ = oracle.macro(p, st.f, st.R)
        ref[m] = (ux, uy, st.R.copy())
    for storage in ("f64", "f32", "f16dev", "bf16dev"):
        err = _sweep_errors(w, storage, w.beads(), ref)
        for m in marks:
            eu, er, _ = err[m]
            print(f"[precision sweep] {storage} step {m}: velocity err {eu:.3e} U, "
                  f"bead err {er:.3e} lu", flush=True)
            if m < 20000 or storage in ("f64", "f32"):
                bu, br = SWEEP_BOUNDS[storage]
                assert eu <= bu and er <= br, (storage, m, eu, er)

    # the flip at 20k steps: six starts shifted along x by k * 1e-7 lu
    flips = {s: [] for s in FLIP_BOUNDS}
    for k in range(6):
        R0 = w.beads().copy()
        R0[:, 0] += k * 1e-7
        if k == 0:
            start_ref = {20000: ref[20000]}   # the oracle
        else:
            start_ref = {20000: _sweep_errors(w, "f64", R0, {20000: ref[20000]})[20000][2]}
        for storage in FLIP_BOUNDS:
            eu, er, _ = _sweep_errors(w, storage, R0, start_ref)[20000]
            print(f"[precision flip] {storage} start +{k}e-7: velocity err {eu:.3e} U, "
                  f"bead err {er:.3e} lu", flush=True)
            flips[storage].append((eu, er))
    for storage, ((mu, xu), (mr, xr)) in FLIP_BOUNDS.items():
        eu = np.array([e[0] for e in flips[storage]])
        er = np.array([e[1] for e in flips[storage]])
        assert np.median(eu) <= mu and eu.max() <= xu, (storage, eu)
        assert np.median(er) <= mr and er.max() <= xr, (storage, er)
