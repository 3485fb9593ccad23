"""Pins of the oracle's MRT collision (no GPU).

The collision itself is not printed in the paper (Sec. II.C defers the MRT formulation to
its refs [41,44]); these tests pin the oracle's reading against facts fixed by the
mathematics:
  * the moment basis is orthogonal with the known row norms;
  * its equilibrium moments equal the moments of the textbook D2Q9 equilibrium;
  * with every rate equal to 1/tau the MRT step reduces to the textbook BGK step with
    Guo's forcing (a special case that must hold exactly);
  * mass is conserved and momentum gains exactly the force (Guo forcing).
"""
import numpy as np
import pytest

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def textbook_feq(rho, ux, uy):
    eu = EX * ux + EY * uy
    return W * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (ux * ux + uy * uy))


def textbook_bgk_guo(f, tau, Fx, Fy):
    """BGK with Guo's forcing (Guo, Zheng & Shi 2002), written from the textbook."""
    rho = f.sum()
    ux = (f @ EX + 0.5 * Fx) / rho
    uy = (f @ EY + 0.5 * Fy) / rho
    eu = EX * ux + EY * uy
    G = W * ((3 * (EX - ux) + 9 * eu * EX) * Fx + (3 * (EY - uy) + 9 * eu * EY) * Fy)
    return f - (f - textbook_feq(rho, ux, uy)) / tau + (1 - 0.5 / tau) * G


def moment_matrix(orc):
    return np.stack([orc.moments(np.eye(9)[k]) for k in range(9)], axis=1)


def test_basis_orthogonal_with_known_norms(orc):
    M = moment_matrix(orc)
    assert np.array_equal(M @ M.T, np.diag([9.0, 36, 36, 6, 12, 6, 12, 4, 4]))
    # rows: density, momentum x, momentum y are the conserved moments
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[3], EX) and np.array_equal(M[5], EY)


def test_inverse_moments_roundtrip(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        f = rng.uniform(0.01, 0.5, 9)
        assert np.allclose(orc.inverse_moments(orc.moments(f)), f, rtol=0, atol=1e-15)


@pytest.mark.parametrize("rho,ux,uy", [(1.0, 0.0, 0.0), (1.03, 0.05, -0.02), (0.97, -0.1, 0.08)])
def test_equilibrium_moments_match_textbook_equilibrium(orc, rho, ux, uy):
    m_from_feq = orc.moments(textbook_feq(rho, ux, uy))
    assert np.allclose(orc.meq(rho, ux, uy), m_from_feq, rtol=0, atol=1e-15)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.0, 3.0])
def test_mrt_with_equal_rates_is_bgk_with_guo_forcing(orc, tau):
    rng = np.random.default_rng(int(tau * 100))
    for _ in range(10):
        f = textbook_feq(1.0 + rng.uniform(-0.05, 0.05), *rng.uniform(-0.05, 0.05, 2))
        f = f * (1 + rng.uniform(-0.05, 0.05, 9))
        Fx, Fy = rng.uniform(-1e-3, 1e-3, 2)
        s = 1.0 / tau
        got = orc.collide(f, s, s, s, s, Fx, Fy)
        assert np.allclose(got, textbook_bgk_guo(f, tau, Fx, Fy), rtol=0, atol=5e-16)


def test_collision_conserves_mass_and_adds_force(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        f = rng.uniform(0.01, 0.5, 9)
        Fx, Fy = rng.uniform(-0.01, 0.01, 2)
        s_nu = rng.uniform(0.1, 1.9)
        out = orc.collide(f, s_nu, 1.64, 1.54, 8 * (2 - s_nu) / (8 - s_nu), Fx, Fy)
        assert abs(out.sum() - f.sum()) <= 2e-15 * f.sum()
        assert abs(out @ EX - (f @ EX + Fx)) <= 2e-15
        assert abs(out @ EY - (f @ EY + Fy)) <= 2e-15


def test_equilibrium_is_a_fixed_point(orc):
    f = textbook_feq(1.0, 0.03, -0.01)
    out = orc.collide(f, 0.7, 1.64, 1.54, 1.2, 0.0, 0.0)
    assert np.allclose(out, f, rtol=0, atol=1e-16)


def test_stream_is_a_permutation_plus_wall_terms(orc):
    """Streaming with U = 0 only moves values: the multiset is preserved and mass too."""
    p = orc.OracleParams(nx=7, ny=5, u_wall=0.0)
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, (9, 5, 7))
    g = orc.stream(p, f)
    assert np.array_equal(np.sort(f.ravel()), np.sort(g.ravel()))
    # a population at an interior node moves by e_k (periodic in x)
    for k in range(9):
        j, i = 2, 3
        assert g[k, j + int(EY[k]), (i + int(EX[k])) % 7] == f[k, j, i]
    # a population leaving through the bottom wall comes back reversed at the same node
    opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
    for k in (4, 7, 8):
        assert g[opp[k], 0, 3] == f[k, 0, 3]


def test_moving_wall_term(orc):
    """Reflected populations pick up 6 w rho0 e.u_w: the wall momentum transfer."""
    U = 0.02
    p = orc.OracleParams(nx=4, ny=3, u_wall=U)
    f = np.zeros((9, 3, 4))
    f[7, 0, 1] = 1.0        # (-1,-1) leaving through the bottom wall (u_w = -U)
    f[5, 2, 1] = 1.0        # (1,1) leaving through the top wall (u_w = +U)
    g = orc.stream(p, f)
    assert g[5, 0, 1] == pytest.approx(1.0 + 6 * (1 / 36) * (1 * -U), abs=1e-17)
    assert g[7, 2, 1] == pytest.approx(1.0 + 6 * (1 / 36) * (-1 * U), abs=1e-17)
