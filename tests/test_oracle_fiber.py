"""Pins of the oracle's fiber coupling (no GPU).

  * Eq. (2): phi = 1/2 exactly on the bead surface |r - R| = a, and the lattice sum of
    phi matches the Sommerfeld expansion pi a^2 + pi^3 xi^2 / 12 of the continuous
    integral;
  * Eq. (4): spreading conserves the total force, sum_x f(x) = sum_i F_i;
  * Eqs. (10)-(12): the forces are minus the gradient of the stretching energy plus the
    bending energy -k_b sum t_{j+1}.t_j (checked by central finite differences), sum to
    zero, carry no torque, and vanish for a straight fiber at rest length;
  * the coupled step (Sec. II.C) keeps the point symmetry of a fiber centred in the
    channel, leaves a quiescent fluid with an unstressed fiber at rest, and conserves
    mass.
"""
import ctypes
import ctypes.util
import math

import numpy as np
import pytest

import workloads


def params(orc, **kw):
    base = dict(nx=40, ny=30, u_wall=0.0, nu_f=0.1, eta_ratio=50.0, xi=1.0, n_beads=1,
                radius=2.0, l0=4.0, k_s=1.0, k_b=0.1)
    base.update(kw)
    return orc.OracleParams(**base)


def test_tanh_saturates_to_minus_one_in_double():
    """The oracle skips rows where phi is exactly zero; that rests on tanh(t) == -1.0
    for t <= -20 in the C library it links."""
    libm = ctypes.CDLL(ctypes.util.find_library("m"))
    libm.tanh.restype = ctypes.c_double
    libm.tanh.argtypes = [ctypes.c_double]
    for t in np.linspace(20.0, 60.0, 4001):
        assert libm.tanh(-t) == -1.0
    assert libm.tanh(-19.0) != -1.0


def test_phi_is_half_on_the_surface(orc):
    p = params(orc, radius=2.0, xi=0.7)
    # node (10, 10) has its centre at (10.5, 10.5); put the bead 2.0 to its left
    assert orc.phi(p, 8.5, 10.5, 10, 10) == 0.5
    assert orc.phi(p, 10.5, 10.5, 10, 10) == pytest.approx(0.5 * (math.tanh(2.0 / 0.7) + 1))


def test_phi_minimum_image_in_x(orc):
    p = params(orc, nx=40)
    assert orc.phi(p, 0.5, 10.5, 39, 10) == orc.phi(p, 0.5, 10.5, 1, 10)
    assert orc.phi(p, 40.5, 10.5, 0, 10) == orc.phi(p, 0.5, 10.5, 0, 10)


@pytest.mark.parametrize("a,xi,tol", [(2.0, 1.0, 5e-3), (3.0, 1.0, 1e-3), (4.0, 1.0, 1e-3), (4.0, 0.5, 3e-3)])
def test_lattice_sum_of_phi_matches_sommerfeld(orc, a, xi, tol):
    p = params(orc, nx=64, ny=64, radius=a, xi=xi)
    rng = np.random.default_rng(int(a * 10))
    for _ in range(3):
        R = np.array([[32 + rng.uniform(0, 1), 32 + rng.uniform(0, 1)]])
        A = orc.fields(p, R)[0][0]
        expect = math.pi * a * a + math.pi ** 3 * xi * xi / 12
        assert abs(A - expect) <= tol * expect


def test_force_spreading_conserves_total_force(orc):
    w = workloads.c1_small_fp64()
    p = orc.OracleParams.from_mapping(w.params())
    R = w.beads() + workloads.perturbation((5, 2), 0.3, seed=11)
    A, F, eta, fx, fy = orc.fields(p, R)
    assert abs(F[:, 0].sum()) < 1e-15 * np.abs(F).max() * 10
    # with the forces made non-zero-sum the spread field still carries exactly sum F
    assert fx.sum() == pytest.approx(F[:, 0].sum(), abs=1e-15 * np.abs(F).sum())
    assert fy.sum() == pytest.approx(F[:, 1].sum(), abs=1e-15 * np.abs(F).sum())
    assert np.all(eta >= p.nu_f - 1e-18)


def energy(R, ks, kb, l0):
    """Stretching energy of Eq. (9) plus the bending energy -k_b sum_j t_{j+1}.t_j."""
    d = np.diff(R, axis=0)
    L = np.linalg.norm(d, axis=1)
    t = d / L[:, None]
    return (ks / (2 * l0 * l0)) * np.sum((L - l0) ** 2) - kb * np.sum(np.sum(t[1:] * t[:-1], axis=1))


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 9])
def test_forces_are_minus_gradient_of_energy(orc, N):
    ks, kb, l0 = 3.0, 0.7, 4.0
    p = params(orc, n_beads=N, k_s=ks, k_b=kb, l0=l0)
    rng = np.random.default_rng(N)
    R = workloads.straight_fiber(N, l0, 0.3, 20.0, 15.0) + rng.uniform(-0.8, 0.8, (N, 2))
    F = orc.bead_forces(p, R)
    h = 1e-6
    G = np.zeros_like(R)
    for i in range(N):
        for c in range(2):
            Rp = R.copy(); Rp[i, c] += h
            Rm = R.copy(); Rm[i, c] -= h
            G[i, c] = -(energy(Rp, ks, kb, l0) - energy(Rm, ks, kb, l0)) / (2 * h)
    assert np.allclose(F, G, rtol=0, atol=1e-7 * max(1.0, np.abs(G).max()))
    # internal forces: no net force, no net torque
    assert np.abs(F.sum(axis=0)).max() < 1e-13
    torque = np.sum(R[:, 0] * F[:, 1] - R[:, 1] * F[:, 0])
    assert abs(torque) < 1e-12


def test_squared_cosine_energy_is_not_what_the_forces_derive_from(orc):
    """Eq. (9) prints the bending energy squared in the cosine; the printed forces
    (12a-e) are the gradient of the linear form instead (this is the reading taken)."""
    N, ks, kb, l0 = 5, 0.0, 1.0, 4.0
    p = params(orc, n_beads=N, k_s=ks, k_b=kb, l0=l0)
    R = workloads.straight_fiber(N, l0, 0.0, 20.0, 15.0)
    R[2, 1] += 1.0
    F = orc.bead_forces(p, R)

    def e_sq(R):
        d = np.diff(R, axis=0)
        t = d / np.linalg.norm(d, axis=1)[:, None]
        return -kb * np.sum(np.sum(t[1:] * t[:-1], axis=1) ** 2)

    h = 1e-6
    G = np.zeros_like(R)
    for i in range(N):
        for c in range(2):
            Rp = R.copy(); Rp[i, c] += h
            Rm = R.copy(); Rm[i, c] -= h
            G[i, c] = -(e_sq(Rp) - e_sq(Rm)) / (2 * h)
    assert np.abs(F - G).max() > 1e-3


def test_straight_fiber_at_rest_length_has_no_force(orc):
    N = 6
    p = params(orc, n_beads=N, k_s=5.0, k_b=0.3, l0=4.0)
    R = workloads.straight_fiber(N, 4.0, 0.0, 20.0, 15.0)
    assert np.array_equal(orc.bead_forces(p, R), np.zeros((N, 2)))
    R = workloads.straight_fiber(N, 4.0, 0.7, 20.0, 15.0)
    assert np.abs(orc.bead_forces(p, R)).max() < 1e-14


def test_centred_fiber_keeps_point_symmetry(orc):
    """A fiber centred in the +-U Couette channel maps onto itself under the rotation by
    180 degrees about the centre, so R_i + R_{N+1-i} = 2c at all times."""
    w = workloads.c1_small_fp64()
    p = orc.OracleParams.from_mapping(w.params())
    st = orc.make_state(p, 1, w.beads())
    traj = orc.run(st, 1000, trajectory=True)
    c = np.array([w.cx, w.cy])
    s = traj + traj[:, ::-1, :]
    assert np.abs(s - 2 * c).max() < 1e-11
    # the fiber actually moves (tumbles clockwise in this shear)
    d0 = w.beads()[-1] - w.beads()[0]
    d1 = st.R[-1] - st.R[0]
    assert math.atan2(d1[1], d1[0]) < math.atan2(d0[1], d0[0]) - 1e-3


def test_quiescent_fluid_with_unstressed_fiber_stays_at_rest(orc):
    N = 4
    p = params(orc, n_beads=N, k_s=5.0, k_b=0.3, l0=4.0, u_wall=0.0)
    R = workloads.straight_fiber(N, 4.0, 0.0, 20.0, 15.0)
    st = orc.make_state(p, 0, R)
    f0 = st.f.copy()
    orc.run(st, 100)
    assert np.abs(st.f - f0).max() < 1e-15
    assert np.abs(st.R - R).max() < 1e-13


def test_bead_velocity_of_uniform_flow_is_that_flow(orc):
    """Eq. (5) is a phi-weighted mean: in a uniform stream the beads move with it."""
    p = params(orc, n_beads=1, nx=32, ny=32, u_wall=0.0)
    st = orc.make_state(p, 0, np.array([[16.3, 15.8]]))
    # a uniform stream along x at rest density: shift every node to equilibrium at u
    EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1.0])
    W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    u = 1e-3
    feq = W * (1 + 3 * EX * u + 4.5 * (EX * u) ** 2 - 1.5 * u * u)
    st.f[:] = feq[:, None, None]
    orc.run(st, 1)
    assert st.V[0, 0] == pytest.approx(u, rel=1e-3)


def spring_energy(R, ks, l0):
    L = np.linalg.norm(np.diff(R, axis=0), axis=1)
    return (ks / (2 * l0 * l0)) * np.sum((L - l0) ** 2)


def test_spring_modes_dissipate_in_quiescent_fluid(orc):
    """With no driving, the overdamped chain must lose spring energy: the coupling of
    Eqs. (4),(5) through the viscous fluid is dissipative.  This pins the reading of the
    velocity field in Eq. (5) as Guo's macroscopic velocity (j + f/2)/rho; with the bare
    momentum j/rho the stretch modes of overlapping beads grow instead."""
    w = workloads.c1_small_fp64().with_(u_wall=0.0)
    p = orc.OracleParams.from_mapping(w.params())
    R = w.beads().copy()
    d = np.array([math.cos(math.pi / 4), math.sin(math.pi / 4)])
    R[0] -= 0.2 * d; R[4] += 0.2 * d; R[1] += 0.1 * d; R[3] -= 0.1 * d
    st = orc.make_state(p, 0, R)
    e = [spring_energy(st.R, p.k_s, p.l0)]
    for _ in range(6):
        orc.run(st, 100)
        e.append(spring_energy(st.R, p.k_s, p.l0))
    assert e[1] < 0.1 * e[0]
    assert max(e[1:]) < 0.1 * e[0] and e[-1] < 1e-3 * e[0]
