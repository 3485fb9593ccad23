"""Several fibers (the outlook of Sec. V applied to the chain of Sec. II.B): beads
c L .. c L + L - 1 form fiber c; springs and bending act inside a fiber only. By default
fibers interact through the fluid alone (the paper gives no excluded-volume force); an
optional pair repulsion between beads of different fibers, (k/2)(d - r)^2 for r < d,
can be switched on.

Pins: the forces on a set of fibers are exactly those of each fiber alone; two fibers
placed point-symmetrically about the centre of the +-U Couette channel stay
point-symmetric (the rotation by 180 degrees maps the problem onto itself, swapping the
fibers and reversing their bead order); the repulsion is minus the gradient of its
energy, has no net force or torque, acts between fibers only and within range, and
across the periodic boundary.
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


# ---------------------------------------------------------------- excluded volume ----

def ev_params(**kw):
    base = dict(nx=120, ny=80, u_wall=0.0, nu_f=0.1, eta_ratio=20.0, xi=1.0, n_beads=6,
                radius=2.0, l0=4.0, k_s=0.0, k_b=0.0, n_chains=2, ev_k=0.3, ev_range=0.0)
    base.update(kw)
    return oracle.OracleParams(**base)


def ev_energy(p, R):
    """(k/2) sum over pairs of beads of different fibers closer than d of (d - r)^2,
    with the minimum image in x (a direct sum over unordered pairs)."""
    d = p.ev_range if p.ev_range > 0 else 2 * p.radius
    L = p.n_beads // p.n_chains
    U = 0.0
    for i in range(p.n_beads):
        for j in range(i + 1, p.n_beads):
            if i // L == j // L:
                continue
            dx = R[i, 0] - R[j, 0]
            dx -= p.nx * round(dx / p.nx)
            r = math.hypot(dx, R[i, 1] - R[j, 1])
            if r < d:
                U += 0.5 * p.ev_k * (d - r) ** 2
    return U


def two_close_fibers(dy=3.1, x0=30.0):
    a = workloads.straight_fiber(3, 4.0, 0.0, x0, 40.0)
    b = workloads.straight_fiber(3, 4.0, 0.15, x0 + 1.3, 40.0 + dy)
    return np.concatenate([a, b])


def test_excluded_volume_is_minus_the_gradient_of_its_energy():
    p = ev_params()
    R = two_close_fibers()
    F = oracle.bead_forces(p, R)
    h = 1e-6
    for b in range(p.n_beads):
        for c in range(2):
            Rp, Rm = R.copy(), R.copy()
            Rp[b, c] += h
            Rm[b, c] -= h
            g = (ev_energy(p, Rp) - ev_energy(p, Rm)) / (2 * h)
            assert abs(F[b, c] + g) <= 1e-7 * max(1.0, abs(g))
    assert np.abs(F).max() > 1e-2                       # the fibers do overlap
    assert np.abs(F.sum(axis=0)).max() < 1e-14           # pairwise: no net force
    torque = np.sum(R[:, 0] * F[:, 1] - R[:, 1] * F[:, 0])
    assert abs(torque) < 1e-12


def test_excluded_volume_acts_between_fibers_only_and_within_range():
    R = two_close_fibers()
    # one fiber of six beads: the beads of a fiber never repel each other
    assert np.array_equal(oracle.bead_forces(ev_params(n_chains=1), R),
                          oracle.bead_forces(ev_params(n_chains=1, ev_k=0.0), R))
    # fibers farther apart than d feel nothing; a larger range reaches them
    far = two_close_fibers(dy=4.5)
    assert np.abs(oracle.bead_forces(ev_params(), far)).max() == 0.0
    assert np.abs(oracle.bead_forces(ev_params(ev_range=5.0), far)).max() > 0.0


def test_excluded_volume_uses_the_minimum_image():
    p = ev_params()
    a = workloads.straight_fiber(3, 4.0, 0.0, 4.0, 40.0)        # beads at x = 0, 4, 8
    b = workloads.straight_fiber(3, 4.0, 0.0, p.nx - 5.0, 40.5)  # beads at x = nx - 9 .. nx - 1
    R = np.concatenate([a, b])
    F = oracle.bead_forces(p, R)
    # bead 0 (x = 0) and bead 5 (x = nx - 1) are 1 apart through the periodic boundary
    assert F[0, 0] > 0 and F[5, 0] < 0
    assert np.abs(F.sum(axis=0)).max() < 1e-14


def test_excluded_volume_pushes_overlapping_fibers_apart():
    R = two_close_fibers(dy=2.0)
    gaps = []
    for k in (0.0, 0.05):
        p = ev_params(ev_k=k, k_s=0.05 * 16.0, k_b=0.01)
        st = oracle.make_state(p, 0, R)
        oracle.run(st, 400)
        gaps.append(np.mean(st.R[3:, 1]) - np.mean(st.R[:3, 1]))
    assert gaps[1] > gaps[0] + 0.05
