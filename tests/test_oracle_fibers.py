"""Several fibers (the survey's NEXT-4 widening of Sec. II.B): beads c L .. c L + L - 1
form fiber c; springs and bending act inside a fiber only, and fibers interact through
the fluid alone (the paper gives no excluded-volume force, so none is modelled).

Pins: the forces on a set of fibers are exactly those of each fiber alone; and two
fibers placed point-symmetrically about the centre of the +-U Couette channel stay
point-symmetric (the rotation by 180 degrees maps the problem onto itself, swapping the
fibers and reversing their bead order).
"""
import math

import numpy as np

import oracle
import workloads


def test_forces_of_several_fibers_are_those_of_each_fiber_alone():
    rng = np.random.default_rng(5)
    L, C = 6, 3
    R = np.concatenate([workloads.straight_fiber(L, 3.0, rng.uniform(0, math.pi),
                                                 20 + 25 * c, 30) for c in range(C)])
    R += rng.normal(0, 0.4, R.shape)                  # bent and stretched
    base = dict(nx=100, ny=60, n_beads=L * C, l0=3.0, k_s=1.3, k_b=0.4, fx_ext=1e-4)
    F = oracle.bead_forces(oracle.OracleParams(**base, n_chains=C), R)
    for c in range(C):
        one = oracle.OracleParams(**{**base, "n_beads": L})
        Fc = oracle.bead_forces(one, R[c * L:(c + 1) * L])
        assert np.array_equal(F[c * L:(c + 1) * L], Fc)
    # one fiber of all beads would couple the last bead of a fiber to the next fiber
    F1 = oracle.bead_forces(oracle.OracleParams(**base), R)
    assert np.abs(F1 - F).max() > 1e-3


def test_two_fibers_keep_the_point_symmetry_of_the_channel():
    nx, ny, L = 64, 40, 4
    c = np.array([nx / 2, ny / 2])
    A = workloads.straight_fiber(L, 2.0, 0.5, c[0] - 12.0, c[1] + 5.0)
    B = 2 * c - A[::-1]                               # the rotated image, reversed order
    p = oracle.OracleParams(nx=nx, ny=ny, u_wall=0.01, nu_f=0.05, eta_ratio=20.0, xi=1.0,
                            n_beads=2 * L, radius=1.0, l0=2.0, k_s=0.3, k_b=2e-3,
                            n_chains=2)
    st = oracle.make_state(p, 1, np.concatenate([A, B]))
    traj = oracle.run(st, 400, trajectory=True)
    sym = traj[:, :L] + traj[:, L:][:, ::-1]
    assert np.abs(sym - 2 * c).max() < 1e-11
    assert np.abs(traj[-1] - traj[0]).max() > 1e-2     # the fibers do move
