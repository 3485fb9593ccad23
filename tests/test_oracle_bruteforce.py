"""Brute force: the oracle's coupled step against a second formulation written here in
numpy on tiny lattices (8 x 6 and 6 x 5, two or three beads, 50 steps).

The second formulation shares the oracle's reading of the paper (Sec. II.C, Eqs. (1)-(5),
the MRT step with Guo forcing and moving-wall bounce-back) but none of its arrangement:
  * the moment matrix M of the Lallemand-Luo basis is written out as a 9 x 9 array and
    inverted numerically (the oracle uses M^T with the row norms);
  * equilibria are built as populations from the second-order Maxwellian and mapped to
    moments through M, and the Guo source as populations, w_k [3 (e_k - u) + 9 (e_k . u)
    e_k] . f, also mapped through M (the oracle writes both directly in moment space);
  * phi, A_i and the force density are dense sums over every node with the minimum image
    and no cutoff (Eqs. (1)-(4));
  * streaming shifts whole arrays (np.roll) and then overwrites the wall rows with the
    halfway bounce-back of the reflected population plus 6 w_k (e_k . u_wall);
  * Eq. (5) averages Guo's velocity (j + f/2)/rho after the step with phi and A_i of the
    step's start, and the beads move by forward Euler.
Bead forces are taken from the oracle (pinned on their own against minus the gradient of
the energy).  A transposed operand, a wrong sign of the wall term, a swapped direction or a
force applied at the wrong time level changes the result far beyond the 1e-13 tolerance
(summation order alone); four such mistakes planted in the second formulation (the wall
term's sign, the (I - S/2) factor of the source, the half force in Eq. (5), phi at the
new positions) are each seen.
"""
import math

import numpy as np
import pytest

import oracle

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
M = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],          # rho
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],     # e
    [4, -2, -2, -2, -2, 1, 1, 1, 1],      # epsilon
    [0, 1, 0, -1, 0, 1, -1, -1, 1],       # j_x
    [0, -2, 0, 2, 0, 1, -1, -1, 1],       # q_x
    [0, 0, 1, 0, -1, 1, 1, -1, -1],       # j_y
    [0, 0, -2, 0, 2, 1, 1, -1, -1],       # q_y
    [0, 1, -1, 1, -1, 0, 0, 0, 0],        # p_xx
    [0, 0, 0, 0, 0, 1, -1, 1, -1],        # p_xy
], dtype=float)
MINV = np.linalg.inv(M)


def feq(rho, ux, uy):
    eu = E[:, 0, None, None] * ux + E[:, 1, None, None] * uy
    return W[:, None, None] * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux ** 2 + uy ** 2))


def guo(ux, uy, fx, fy):
    ex, ey = E[:, 0, None, None], E[:, 1, None, None]
    eu = ex * ux + ey * uy
    return W[:, None, None] * (3 * ((ex - ux) * fx + (ey - uy) * fy) + 9 * eu * (ex * fx + ey * fy))


def phi_dense(p, R):
    """phi_i at every node centre (x + 1/2, y + 1/2), minimum image in x: [N, ny, nx]."""
    x = np.arange(p.nx) + 0.5
    y = np.arange(p.ny) + 0.5
    out = []
    for Rx, Ry in R:
        dx = x - Rx
        dx = dx - p.nx * np.floor(dx / p.nx + 0.5)
        dy = y - Ry
        r = np.sqrt(dx[None, :] ** 2 + dy[:, None] ** 2)
        out.append(0.5 * (np.tanh((p.radius - r) / p.xi) + 1.0))
    return np.array(out)


def step(p, f, R, plant=None):
    F = oracle.bead_forces(p, R)
    ph = phi_dense(p, R)
    A = ph.sum(axis=(1, 2))
    sphi = ph.sum(axis=0)
    fx = np.einsum("i,iyx->yx", F[:, 0] / A, ph)
    fy = np.einsum("i,iyx->yx", F[:, 1] / A, ph)
    nu = p.nu_f * (1 + (p.eta_ratio - 1) * sphi)
    s_nu = 1 / (3 * nu + 0.5)
    s_q = 8 * (2 - s_nu) / (8 - s_nu)
    # collision in moment space, node by node through M
    rho = f.sum(axis=0)
    jx = np.einsum("k,kyx->yx", E[:, 0].astype(float), f)
    jy = np.einsum("k,kyx->yx", E[:, 1].astype(float), f)
    ux, uy = (jx + fx / 2) / rho, (jy + fy / 2) / rho
    m = np.einsum("ak,kyx->ayx", M, f)
    meq = np.einsum("ak,kyx->ayx", M, feq(rho, ux, uy))
    src = np.einsum("ak,kyx->ayx", M, guo(ux, uy, fx, fy))
    S = np.zeros((9,) + rho.shape)
    S[1], S[2], S[4], S[6], S[7], S[8] = p.s_e, p.s_eps, s_q, s_q, s_nu, s_nu
    if plant == "no_half_rate_on_source":
        mstar = m - S * (m - meq) + src
    else:
        mstar = m - S * (m - meq) + (1 - S / 2) * src
    fpost = np.einsum("ka,ayx->kyx", MINV, mstar)
    # push streaming, periodic in x; wall rows then take the reflected population
    fn = np.empty_like(fpost)
    for k in range(9):
        fn[k] = np.roll(fpost[k], shift=(E[k, 1], E[k, 0]), axis=(0, 1))
    U = -p.u_wall if plant == "wall_sign" else p.u_wall
    for k in range(9):
        if E[k, 1] == 1:     # arrives at the bottom row from below the wall at y = 0
            fn[k, 0] = fpost[OPP[k], 0] + 6 * W[k] * (E[k, 0] * -U)
        if E[k, 1] == -1:    # arrives at the top row from above the wall at y = ny
            fn[k, -1] = fpost[OPP[k], -1] + 6 * W[k] * (E[k, 0] * U)
    # Eq. (5) with phi^n, A^n and Guo's velocity after the step
    rho1 = fn.sum(axis=0)
    half = 0.0 if plant == "bare_velocity" else 0.5
    vx = (np.einsum("k,kyx->yx", E[:, 0].astype(float), fn) + half * fx) / rho1
    vy = (np.einsum("k,kyx->yx", E[:, 1].astype(float), fn) + half * fy) / rho1
    if plant == "phi_after_move":  # Eq. (5) with phi at the new positions instead of phi^n
        ph = phi_dense(p, R + 1e-3)
    V = np.stack([(ph * vx).sum(axis=(1, 2)), (ph * vy).sum(axis=(1, 2))], axis=1) / A[:, None]
    return fn, R + V


CASES = [
    (8, 6, [(2.3, 2.9), (4.1, 3.4)], 0.02),
    (6, 5, [(1.2, 2.4), (2.9, 2.6), (4.4, 2.2)], -0.015),
]


def both(nx, ny, R, u, plant=None, steps=50):
    R = np.array(R, dtype=float)
    p = oracle.OracleParams(nx=nx, ny=ny, u_wall=u, nu_f=0.09, eta_ratio=20.0, xi=0.5,
                            n_beads=len(R), radius=0.8, l0=1.7, k_s=0.05, k_b=0.01)
    rng = np.random.default_rng(nx * 100 + ny)
    f0 = oracle.init(p, 1) + 1e-3 * rng.standard_normal((9, ny, nx))
    st = oracle.make_state(p, 1, R)
    st.f[:] = f0
    oracle.run(st, steps)
    f, Rb = f0.copy(), R.copy()
    for _ in range(steps):
        f, Rb = step(p, f, Rb, plant)
    return f, Rb, st, R


@pytest.mark.parametrize("nx,ny,R,u", CASES)
def test_oracle_equals_second_formulation(nx, ny, R, u):
    f, Rb, st, R0 = both(nx, ny, R, u)
    assert np.max(np.abs(f - st.f) / np.abs(st.f)) < 1e-13
    # positions of a few lattice units: 1e-13 relative
    assert np.max(np.abs(Rb - st.R)) < 1e-13 * np.max(np.abs(st.R))
    assert np.max(np.abs(Rb - R0)) > 1e-4      # the beads did move


@pytest.mark.parametrize("plant", ["wall_sign", "no_half_rate_on_source", "bare_velocity",
                                   "phi_after_move"])
def test_a_planted_mistake_is_seen(plant):
    f, Rb, st, _ = both(*CASES[0], plant=plant, steps=20)
    err = max(np.max(np.abs(f - st.f) / np.abs(st.f)), np.max(np.abs(Rb - st.R)))
    assert err > 1e-8


def test_second_formulation_basics():
    # the inverse is the textbook one: M M^T is diagonal with the row norms
    assert np.allclose(M @ M.T, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]))
    assert np.allclose(MINV, M.T / np.array([9, 36, 36, 6, 12, 6, 12, 4, 4]))
    # the Guo source carries the force and no mass: moments (0, ., ., fx, ., fy, ...)
    ux, uy, fx, fy = (np.full((1, 1), v) for v in (0.03, -0.02, 1e-3, 2e-3))
    m = np.einsum("ak,kyx->ayx", M, guo(ux, uy, fx, fy))[:, 0, 0]
    assert abs(m[0]) < 1e-18 and math.isclose(m[3], 1e-3) and math.isclose(m[5], 2e-3)
