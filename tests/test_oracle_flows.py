"""Pins of the oracle's lattice Boltzmann stage against closed-form flows (no GPU).

  * steady Couette between walls moving at -U and +U: u_x = U (2y/H - 1) (Sec. IV.A);
  * Couette start-up from rest: Fourier-series solution of the diffusion equation;
  * the paper's sandwich benchmark (Sec. III.A, Eqs. (13),(14)): with a smooth viscosity
    eta(y) the steady shear stress is uniform, so v(y) is fixed by int_0^y 1/eta exactly;
  * body-force Poiseuille flow, which is reproduced exactly by the MRT scheme with the
    magic heat-flux rate and Guo forcing.
"""
import math

import numpy as np
import pytest


def run_fields(orc, p, f, snu, fx, fy, steps):
    for _ in range(steps):
        f = orc.lbm_step_fields(p, f, snu, fx, fy)
    return f


def ux_profile(orc, p, f, fx=0.0):
    rho, vx, _ = orc.bare_velocity(p, f)
    return (vx * rho + 0.5 * fx) / rho


@pytest.mark.parametrize("tau,tol", [(0.6, 5e-7), (3.0, 5e-6)])
def test_steady_couette_default_mrt_rates(orc, tau, tol):
    """Linear profile to within 1e-5 U; the residual is a compressibility effect: its
    relative size scales as U^2 (an error in the walls or streaming would not)."""
    ny = 16
    rel = []
    for U in (0.01, 0.005):
        p = orc.OracleParams(nx=3, ny=ny, u_wall=U, nu_f=(tau - 0.5) / 3)
        st = orc.make_state(p, 1)
        orc.run(st, 3000)
        u = ux_profile(orc, p, st.f)
        y = np.arange(ny) + 0.5
        exact = U * (2 * y / ny - 1)
        rel.append(np.abs(u - exact[:, None]).max() / U)
    assert rel[0] <= tol
    assert 3.5 < rel[0] / rel[1] < 4.5


def test_steady_couette_bgk_rates_is_exact(orc):
    U, ny, tau = 0.01, 16, 0.9
    s = 1 / tau
    p = orc.OracleParams(nx=2, ny=ny, u_wall=U, nu_f=(tau - 0.5) / 3, s_e=s, s_eps=s,
                         s_q_fixed=s)
    st = orc.make_state(p, 0)
    orc.run(st, 6000)
    u = ux_profile(orc, p, st.f)
    y = np.arange(ny) + 0.5
    assert np.abs(u - (U * (2 * y / ny - 1))[:, None]).max() <= 1e-9 * U


def startup_series(U, nu, H, y, t, terms=400):
    eta = y / H
    u = U * (2 * eta - 1)
    for n in range(2, 2 * terms + 1, 2):
        u = u + 4 * U / (n * math.pi) * np.sin(n * math.pi * eta) * math.exp(-nu * (n * math.pi / H) ** 2 * t)
    return u


def test_couette_startup_transient_second_order(orc):
    U, tau = 0.01, 0.8
    nu = (tau - 0.5) / 3
    errs = []
    for ny in (32, 64):
        p = orc.OracleParams(nx=2, ny=ny, u_wall=U, nu_f=nu)
        st = orc.make_state(p, 0)
        t = int(round(0.02 * ny * ny / nu))
        orc.run(st, t)
        u = ux_profile(orc, p, st.f)[:, 0]
        y = np.arange(ny) + 0.5
        errs.append(np.abs(u - startup_series(U, nu, ny, y, t)).max())
    assert errs[0] <= 0.01 * U
    assert errs[0] / errs[1] > 3.0          # second order in the lattice spacing


def sandwich_profile(y, H, xi):
    """phi of Eq. (14) with z_L = H/3, z_R = 2H/3."""
    zl, zr = H / 3, 2 * H / 3
    return np.where(y <= H / 2, 0.5 * (np.tanh((zl - y) / xi) + 1), 0.5 * (np.tanh((y - zr) / xi) + 1))


def test_sandwich_benchmark_matches_integral_of_inverse_viscosity(orc):
    """Sec. III.A: solid | fluid | solid sandwich as a smooth viscosity profile."""
    ny, U, tau_f, r_eta, xi = 48, 0.01, 0.8, 50.0, 0.5
    nu_f = (tau_f - 0.5) / 3
    y = np.arange(ny) + 0.5
    eta = nu_f * (1 + (r_eta - 1) * sandwich_profile(y, ny, xi))
    snu = np.repeat((1 / (3 * eta + 0.5))[:, None], 2, axis=1)
    p = orc.OracleParams(nx=2, ny=ny, u_wall=U, nu_f=nu_f)
    f = orc.init(p, 1)
    zero = np.zeros((ny, 2))
    f = run_fields(orc, p, f, snu, zero, zero, 12000)
    u = ux_profile(orc, p, f)[:, 0]
    # exact steady solution: uniform stress => du/dy = tau / eta(y)
    yy = np.linspace(0, ny, 200001)
    inv = 1 / (nu_f * (1 + (r_eta - 1) * sandwich_profile(yy, ny, xi)))
    cum = np.concatenate([[0], np.cumsum(0.5 * (inv[1:] + inv[:-1]) * np.diff(yy))])
    exact = -U + 2 * U * np.interp(y, yy, cum) / cum[-1]
    assert np.abs(u - exact).max() <= 0.005 * U
    # and the sharp-interface limit Eq. (13) is approached (a few per cent at this xi)
    sharp = np.clip(-U + 2 * U * (y - ny / 3) / (ny / 3), -U, U)
    assert np.abs(u - sharp).max() <= 0.08 * U


def test_body_force_poiseuille_exact_with_magic_rate(orc):
    ny, g, tau = 16, 1e-6, 0.9
    nu = (tau - 0.5) / 3
    p = orc.OracleParams(nx=2, ny=ny, u_wall=0.0, nu_f=nu)
    f = orc.init(p, 0)
    snu = np.full((ny, 2), 1 / tau)
    fx = np.full((ny, 2), g)
    zero = np.zeros((ny, 2))
    f = run_fields(orc, p, f, snu, fx, zero, 8000)
    u = ux_profile(orc, p, f, fx)[:, 0]
    y = np.arange(ny) + 0.5
    exact = g * y * (ny - y) / (2 * nu)
    assert np.abs(u - exact).max() <= 1e-8 * exact.max()


def test_mass_conserved_with_moving_walls(orc):
    import workloads
    w = workloads.c1_small_fp64()
    p = orc.OracleParams.from_mapping(w.params())
    st = orc.make_state(p, 1, w.beads())
    m0 = st.f.sum()
    orc.run(st, 300)
    assert abs(st.f.sum() - m0) <= 1e-13 * 300 * m0


def test_static_profile_in_the_full_step_is_the_sandwich(orc):
    """A fixed profile phi_s(y) in the full step (no beads) is the sandwich of Sec. III.A:
    the same populations as the LBM stage driven with eta(y) directly."""
    ny, U, tau_f, r_eta, xi = 48, 0.01, 0.8, 50.0, 0.5
    nu_f = (tau_f - 0.5) / 3
    y = np.arange(ny) + 0.5
    phi = sandwich_profile(y, ny, xi)
    p = orc.OracleParams(nx=2, ny=ny, u_wall=U, nu_f=nu_f, eta_ratio=r_eta, phi_static=phi)
    st = orc.make_state(p, 1)
    orc.run(st, 400)
    eta = nu_f + (r_eta * nu_f - nu_f) * phi
    snu = np.repeat((1 / (3 * eta + 0.5))[:, None], 2, axis=1)
    zero = np.zeros((ny, 2))
    p0 = orc.OracleParams(nx=2, ny=ny, u_wall=U, nu_f=nu_f)
    f = run_fields(orc, p0, orc.init(p0, 1), snu, zero, zero, 400)
    assert np.abs(st.f - f).max() < 1e-14
