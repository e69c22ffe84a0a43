"""Pins of the FP64 oracle's single-node algebra against what the paper and
the mathematics fix (no GPU).

Each test names the passage of arXiv:1601.04633 it pins.  Nothing here
re-types the oracle's formulas: the expected values come from the velocity
set alone, from textbook identities, or from the polynomial form of the
equilibria written in distribution space.
"""
import math

import numpy as np
import pytest

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


@pytest.fixture(scope="module")
def orc(oracle_mod):
    return oracle_mod.Oracle(8, 1e3, 0.01)


@pytest.fixture(scope="module")
def mats(orc):
    return orc.matrices()


def test_velocity_sets_eq23_eq35(mats):
    """Eq. 23/35 evaluate to rest, the 4 axis and the 4 diagonal links, and
    they equal rows 2-3 of M (Eq. 30) and of N (Eq. 37)."""
    M, _, N, _, e9, e5 = mats
    assert sorted(map(tuple, e9.tolist())) == sorted(
        [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
    np.testing.assert_array_equal(M[1], e9[:, 0])
    np.testing.assert_array_equal(M[2], e9[:, 1])
    np.testing.assert_array_equal(N[1], e5[:, 0])
    np.testing.assert_array_equal(N[2], e5[:, 1])
    np.testing.assert_array_equal(e5, e9[:5])


def test_M_rows_are_lattice_polynomials_eq29_eq30(mats):
    """Eq. 29 names the moments (rho, j, e, p_xx, p_xy, q, eps).  Each row of
    the typed M must be that polynomial of the velocity set (Lallemand & Luo
    moment basis); a typo anywhere in Eq. 30 fails here."""
    M, _, _, _, e9, _ = mats
    ex, ey = e9[:, 0].astype(float), e9[:, 1].astype(float)
    c2 = ex ** 2 + ey ** 2
    rows = [np.ones(9), ex, ey, 3 * c2 - 4, ex ** 2 - ey ** 2, ex * ey,
            (3 * c2 - 5) * ex, (3 * c2 - 5) * ey, (9 * c2 ** 2 - 21 * c2 + 8) / 2]
    np.testing.assert_array_equal(M, np.array(rows))


def test_N_rows_reading_R2_eq37(mats):
    """Eq. 37: rows (1, e_x, e_y, 5|e|^2 - 4, e_x^2 - e_y^2).  The printed last
    row (0,1,-1,1,1) is not orthogonal to the others; the corrected row
    (0,1,-1,1,-1) is e_x^2 - e_y^2."""
    _, _, N, _, _, e5 = mats
    ex, ey = e5[:, 0].astype(float), e5[:, 1].astype(float)
    c2 = ex ** 2 + ey ** 2
    rows = [np.ones(5), ex, ey, 5 * c2 - 4, ex ** 2 - ey ** 2]
    np.testing.assert_array_equal(N, np.array(rows))
    printed = N.copy()
    printed[4] = [0, 1, -1, 1, 1]
    G = printed @ printed.T
    assert np.abs(G - np.diag(np.diag(G))).max() > 0  # printed row is not orthogonal


def test_orthogonality_and_inverses(mats):
    """M M^T = diag(9,6,6,36,4,4,12,12,36), N N^T = diag(5,2,2,20,4); the
    numerically inverted matrices satisfy M M^-1 = I and N N^-1 = I."""
    M, Mi, N, Ni, _, _ = mats
    np.testing.assert_array_equal(M @ M.T, np.diag([9, 6, 6, 36, 4, 4, 12, 12, 36]))
    np.testing.assert_array_equal(N @ N.T, np.diag([5, 2, 2, 20, 4]))
    np.testing.assert_allclose(M @ Mi, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(Mi @ M, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(N @ Ni, np.eye(5), atol=1e-15)
    np.testing.assert_allclose(Ni @ N, np.eye(5), atol=1e-15)


def _feq_poly(drho, u, v, e9, rho0=1.0):
    """Incompressible second-order D2Q9 equilibrium in distribution space
    (deviation form: sums to drho, first moment rho0 u)."""
    eu = e9[:, 0] * u + e9[:, 1] * v
    return W9 * (drho + rho0 * (3 * eu + 4.5 * eu ** 2 - 1.5 * (u * u + v * v)))


def _geq_poly(theta, u, v, a, e5):
    wm = (4 + a) / 20
    w = np.array([(1 - a) / 5] + [wm] * 4)
    cu = e5[:, 0] * u + e5[:, 1] * v
    # moving populations: w theta (1 + c.u / c_sT^2), c_sT^2 = 2 wm (Eq. 43)
    return w * theta * (1 + cu / (2 * wm) * (np.arange(5) > 0))


def test_moment_equilibrium_eq34_reading_R1(mats):
    """M f^eq of the polynomial equilibrium reproduces Eq. 34 exactly, with
    the energy moment -2 drho + 3 rho0 |u|^2 (the printed form lacks the 3)."""
    M, _, _, _, e9, _ = mats
    rng = np.random.default_rng(5)
    for _ in range(10):
        drho, u, v = rng.normal(scale=0.05, size=3)
        m = M @ _feq_poly(drho, u, v, e9)
        uu = u * u + v * v
        expect = [drho, u, v, -2 * drho + 3 * uu, u * u - v * v, u * v, -u, -v, drho - 3 * uu]
        np.testing.assert_allclose(m, expect, atol=1e-16)
        assert abs(m[3] - (-2 * drho + uu)) > 1e-6 or uu < 1e-10   # printed form fails


def test_equilibria_are_fixed_points(oracle_mod, mats):
    """With no force, collision leaves f^eq(drho, u) and g^eq(theta, u)
    unchanged (Eqs. 28, 34, 36, 42).  f^eq, g^eq are built here in
    distribution space, independently of the oracle's moment formulation."""
    _, _, _, _, e9, e5 = mats
    rng = np.random.default_rng(7)
    for a in (-2 / 3, 0.0, 0.5, -3.0):
        o = oracle_mod.Oracle(8, 1e3, 0.01, gbeta_override=0.0, a=a)
        for _ in range(5):
            drho, u, v, th = rng.normal(scale=[0.01, 0.05, 0.05, 0.3])
            feq = _feq_poly(drho, u, v, e9)
            geq = _geq_poly(th, u, v, a, e5)
            fs, gs = o.collide(feq, geq)
            np.testing.assert_allclose(fs, feq, atol=2e-17)
            np.testing.assert_allclose(gs, geq, atol=2e-16)


def test_relaxation_spectrum_eq28_eq31_eq38(oracle_mod, mats):
    """Linearised about rest, collision (no force) has eigenvectors M^-1 e_k
    with eigenvalues 1 - S_k for the non-conserved moments (Eq. 28, S of
    Eq. 31-32), and N^-1 e_k with 1 - Q_k (Eqs. 36, 38)."""
    M, Mi, N, Ni, _, _ = mats
    o = oracle_mod.Oracle(16, 1e4, 0.01, gbeta_override=0.0)
    d = oracle_mod.derive(16, 1e4, 0.01, 0.1)
    S = [0, 1, 1, d["s_nu"], d["s_nu"], d["s_nu"], d["s_q"], d["s_q"], d["s_nu"]]
    Q = [0, d["sigma_k"], d["sigma_k"], d["sigma_e"], d["sigma_nu"]]
    eps = 1e-7
    for k in range(3, 9):
        f = Mi[:, k] * eps
        fs, _ = o.collide(f, np.zeros(5))
        np.testing.assert_allclose(M @ fs, np.eye(9)[k] * eps * (1 - S[k]), atol=1e-22)
    for k in range(3, 5):
        g = Ni[:, k] * eps
        _, gs = o.collide(np.zeros(9), g)
        np.testing.assert_allclose(N @ gs, np.eye(5)[k] * eps * (1 - Q[k]), atol=1e-22)
    # theta-independent heat flux modes relax at sigma_k about theta = 0
    for k in (1, 2):
        g = Ni[:, k] * eps
        _, gs = o.collide(np.zeros(9), g)
        np.testing.assert_allclose(N @ gs, np.eye(5)[k] * eps * (1 - Q[k]), atol=1e-22)


def test_force_moments_eq26_reading_R3(orc, mats):
    """Eq. 26 with p -> rho0 c_s^2: zero mass source and momentum source
    rho0 G, and F equals 3 G.(e_i - u) w_i rho0 (1 + 3 e.u + 4.5 (e.u)^2 -
    1.5 u^2) with the D2Q9 weights (4/9, 1/9, 1/36)."""
    _, _, _, _, e9, _ = mats
    rng = np.random.default_rng(11)
    for _ in range(20):
        Gx, Gy, u, v = rng.normal(scale=0.05, size=4)
        F = orc.force(Gx, Gy, u, v)
        assert abs(F.sum()) < 1e-16
        assert abs(F @ e9[:, 0] - Gx) < 1e-16
        assert abs(F @ e9[:, 1] - Gy) < 1e-16
        eu = e9[:, 0] * u + e9[:, 1] * v
        feq = W9 * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u * u + v * v))
        Fref = 3 * (Gx * (e9[:, 0] - u) + Gy * (e9[:, 1] - v)) * feq
        np.testing.assert_allclose(F, Fref, rtol=1e-14, atol=1e-16)


def test_force_closed_form_buoyancy_only(orc, mats):
    """Moment image of Eq. 26 for a vertical buoyancy G = (0, G):
    (0, 0, G, 3Gv(2-3|u|^2), -Gv(2+3u^2-3v^2), Gu(1-3v^2), 6Guv, -G(1-3u^2),
    -3Gv(2-3|u|^2)), plus the analogous horizontal part by the x<->y mirror."""
    M, _, _, _, _, _ = mats
    rng = np.random.default_rng(13)
    for _ in range(20):
        G, u, v = rng.normal(scale=0.05, size=3)
        uu = u * u + v * v
        expect = [0, 0, G, 3 * G * v * (2 - 3 * uu), -G * v * (2 + 3 * u * u - 3 * v * v),
                  G * u * (1 - 3 * v * v), 6 * G * u * v, -G * (1 - 3 * u * u),
                  -3 * G * v * (2 - 3 * uu)]
        np.testing.assert_allclose(M @ orc.force(0.0, G, u, v), expect, atol=1e-16)


def test_collision_conservation(oracle_mod):
    """A collision with buoyancy conserves drho and theta and changes the
    momentum by exactly rho0 G, G = gbeta (theta - theta_ref) (Eqs. 26-27)."""
    o = oracle_mod.Oracle(16, 1e4, 0.01, theta_ref=0.1)
    d = o.derived()
    rng = np.random.default_rng(17)
    e = o.matrices()[4]
    for _ in range(20):
        f = rng.normal(scale=1e-2, size=9)
        g = rng.normal(scale=1e-1, size=5)
        fs, gs = o.collide(f, g)
        th = g.sum()
        G = d["gbeta"] * (th - 0.1)
        assert abs(fs.sum() - f.sum()) < 1e-16
        assert abs(gs.sum() - g.sum()) < 1e-15
        assert abs(fs @ e[:, 0] - f @ e[:, 0]) < 1e-16
        assert abs(fs @ e[:, 1] - f @ e[:, 1] - G) < 1e-16


def test_heat_flux_moment_relaxes_to_u_theta(oracle_mod):
    """Eq. 42: the heat-flux moments relax towards (u theta, v theta) at
    rate sigma_k; with sigma_k the post-collision flux is exact."""
    o = oracle_mod.Oracle(16, 1e4, 0.01, gbeta_override=0.0)
    d = o.derived()
    sk = d["Q"][1]
    rng = np.random.default_rng(19)
    W = o.matrices()
    N, e9 = W[2], W[4]
    for _ in range(10):
        u, v = rng.normal(scale=0.05, size=2)
        f = _feq_poly(0.0, u, v, e9)
        g = rng.normal(scale=0.1, size=5)
        th = g.sum()
        _, gs = o.collide(f, g)
        n0, n1 = N @ g, N @ gs
        np.testing.assert_allclose(n1[1], n0[1] - sk * (n0[1] - u * th), atol=1e-16)
        np.testing.assert_allclose(n1[2], n0[2] - sk * (n0[2] - v * th), atol=1e-16)
