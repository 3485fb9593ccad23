"""Tumbling analysis (Sec. IV): the orbit quantities and the classifier on series whose
answer is known.

  * Jeffery's orbit, Eq. (19), integrated finely here (fourth-order Runge-Kutta): the
    measured period matches pi (r_c + 1/r_c) / gamma and the fit returns r_c;
  * a fiber that relaxes to a fixed angle is stuck; tumbling fibers whose end-to-end
    length dips to 80 % or 30 % of straight make S-turns or are S-coiled;
  * the oracle's stiff three-bead fiber in the channel tumbles on a Jeffery orbit, with the
    fitted r_c between the geometric one and twice it (a bead chain with a smooth interface
    is thicker than its geometric aspect ratio; the paper fits 0.132 for its 0.1 fiber).
"""
import math

import numpy as np
import pytest

from paper_2212_14153_amd import tumbling


def jeffery_series(gamma, r_c, t_end, dt, theta0=0.3):
    def f(th):
        return tumbling.jeffery_omega(th, gamma, r_c)
    n = int(t_end / dt)
    th = np.empty(n + 1)
    th[0] = theta0
    for i in range(n):
        k1 = f(th[i])
        k2 = f(th[i] + 0.5 * dt * k1)
        k3 = f(th[i] + 0.5 * dt * k2)
        k4 = f(th[i] + dt * k3)
        th[i + 1] = th[i] + dt * (k1 + 2 * k2 + 2 * k3 + k4) / 6
    return np.arange(n + 1) * dt, th


def record_from(t, theta, length):
    L = np.broadcast_to(np.asarray(length, dtype=float), theta.shape)
    return np.stack([t, L * np.cos(theta), L * np.sin(theta), 0 * t, 0 * t], axis=1)


def test_jeffery_orbit_period_and_fit():
    gamma, r_c = 1e-3, 0.2
    T = tumbling.jeffery_period(gamma, r_c)
    t, th = jeffery_series(gamma, r_c, 3.2 * T, 2.0)
    a = tumbling.analyse(record_from(t, th, 30.0), gamma=gamma)
    assert a["period"] == pytest.approx(T, rel=1e-3)
    assert a["r_c_fit"] == pytest.approx(r_c, rel=1e-3)
    assert a["turns"] > 3
    assert tumbling.classify(a, gamma) == "jeffery"
    assert np.all(a["omega"] < 0)                      # clockwise in this shear


def test_stuck_fiber():
    gamma = 1e-3
    t = np.arange(0, 40000.0, 10.0)
    th = 0.4 + 0.6 * np.exp(-t / 2000.0)               # settles at 0.4 rad
    a = tumbling.analyse(record_from(t, th, 30.0), gamma=gamma)
    assert tumbling.classify(a, gamma) == "stuck"


@pytest.mark.parametrize("dip,expect", [(0.8, "s-turn"), (0.3, "s-coiled"), (0.97, "jeffery")])
def test_folding_fibers(dip, expect):
    gamma, r_c = 1e-3, 0.2
    T = tumbling.jeffery_period(gamma, r_c)
    t, th = jeffery_series(gamma, r_c, 2.5 * T, 5.0)
    # the length dips each time the fiber crosses the flow direction
    L = 30.0 * (1 - (1 - dip) * np.exp(-(np.sin(th)) ** 2 / 0.02))
    a = tumbling.analyse(record_from(t, th, L), straight_length=30.0, gamma=gamma)
    assert a["L_min"] == pytest.approx(dip, abs=0.02)
    assert tumbling.classify(a, gamma) == expect


def test_director_angle_is_continuous_and_head_tail_symmetric():
    th = np.linspace(0.2, -7.0, 500)
    ex, ey = np.cos(th), np.sin(th)
    sgn = np.where(np.arange(500) % 3 == 0, -1.0, 1.0)   # head and tail swapped at random
    d = tumbling.director_angle(sgn * ex, sgn * ey)
    assert np.abs(d - th).max() < 1e-12      # th[0] = 0.2 lies in [-pi/2, pi/2]


def test_oracle_stiff_fiber_tumbles_on_a_jeffery_orbit():
    import oracle
    import workloads
    # 3 touching beads (a = 2, l0 = 4, l_c = 12, r_c = 1/3) in a 64 x 40 channel:
    # gamma = 1.5e-3, Re_ps = 0.5, K = 3.3 (rigid), C = 0.3
    n, a, l0, nx, ny, u = 3, 2.0, 4.0, 64, 40, 0.03
    gamma = 2 * u / ny
    lc = n * l0
    nu = gamma * lc * lc / (4 * 0.5)
    p = oracle.OracleParams(nx=nx, ny=ny, u_wall=u, nu_f=nu, eta_ratio=50.0, xi=1.0,
                            n_beads=n, radius=a, l0=l0, k_s=0.1 * math.pi * a * a * l0 * l0,
                            k_b=3.3 * nu * gamma * lc * lc / 2)
    st = oracle.make_state(p, 1, workloads.straight_fiber(n, l0, 1.2, nx / 2, ny / 2))
    steps = 6600
    traj = oracle.run(st, steps, trajectory=True)[::10]
    e = traj[:, -1] - traj[:, 0]
    c = traj.mean(axis=1)
    rec = np.column_stack([np.arange(1, steps + 1)[::10], e[:, 0], e[:, 1], c[:, 0], c[:, 1]])
    an = tumbling.analyse(rec, straight_length=(n - 1) * l0, gamma=gamma)
    assert an["turns"] > 1.0
    assert tumbling.classify(an, gamma) == "jeffery"
    r_geo = 2 * a / lc
    assert r_geo < an["r_c_fit"] < 2 * r_geo


@pytest.mark.parametrize("kappa,conf,re", [(3.3e-5, 0.5, 1.5), (3.3, 0.87, 6.0),
                                           (0.33, 0.3, 0.5)])
def test_shape_diagram_points_have_the_papers_groups(kappa, conf, re):
    """Each shape-diagram run sets K, C and Re_ps of Eq. (18) (C up to rounding H to whole
    nodes), r_c = 0.1 with touching beads, L_x = 25 d, r_eta = 100, xi / d = 0.125, and
    the walls move at +-gamma H / 2."""
    import workloads
    w = workloads.flexible_fiber(kappa, conf, re)
    d = 2 * w.radius
    lc = w.n_beads * w.l0
    gamma = 2 * w.u_wall / w.ny
    assert w.l0 == d and d / lc == pytest.approx(0.1)
    assert gamma == pytest.approx(1.5e-4)
    assert gamma * lc ** 2 / (4 * w.nu_f) == pytest.approx(re)
    assert 2 * w.k_b / (w.nu_f * gamma * lc ** 2) == pytest.approx(kappa)
    assert abs(lc / w.ny - conf) <= lc / w.ny ** 2
    assert w.nx == 25 * d and w.eta_ratio == 100 and w.xi / d == 0.125
    R = w.beads()
    assert np.allclose(R[:, 1], w.ny / 2) and R[:, 0].mean() == pytest.approx(w.nx / 2)


def test_final_angle_and_rotation():
    t = np.arange(5.0)
    th = np.radians([0.0, -60.0, -120.0, -160.0, -160.0])     # clockwise to 20 degrees
    a = tumbling.analyse(record_from(t, th, 10.0))
    assert tumbling.final_angle_deg(a) == pytest.approx(20.0)
    assert tumbling.turned_deg(a) == pytest.approx(-160.0)
