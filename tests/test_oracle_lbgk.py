"""Pins of the oracle's double LBGK scheme (the single-relaxation-time
scheme the paper's introduction contrasts with double MRT).

The LBGK collision is computed in distribution space with the textbook
equilibria; the MRT collision in moment space with M, N and their
numerical inverses.  With every non-conserved rate equal the two must agree
to round-off -- an identity, since M^-1 S M = s I on the non-conserved
subspace and the conserved moments sit at equilibrium -- which pins the
LBGK code against the independently written MRT code.  The viscosity and
diffusivity relations are pinned by decaying periodic modes."""
import math

import numpy as np
import pytest

from test_oracle_closed_forms import _ra_for


def _random_states(rng, count):
    for _ in range(count):
        yield rng.uniform(-0.05, 0.05, 9), rng.uniform(-0.4, 0.4, 5)


@pytest.mark.parametrize("kw", [
    dict(n=64, Ra=1e4, Pr=0.01),
    dict(n=32, Ra=1e5, Pr=0.001, gbeta_override=0.3, theta_ref=0.1),
    dict(n=48, Ra=3e3, Pr=0.05, bc=1, gbeta_override=0.2, force_x=0.05),
    dict(n=256, Ra=5e4, Pr=0.005, a=0.5),
])
def test_lbgk_equals_mrt_with_equal_rates(oracle_mod, kw):
    O = oracle_mod
    lb = O.Oracle(collision=O.LBGK, **kw)
    mr = O.Oracle(collision=O.MRT, **kw)
    d = lb.derived()
    s_nu, sk = d["S"][4], d["Q"][1]
    mr.set_rates([0.0, 1.0, 1.0] + [s_nu] * 6, [0.0] + [sk] * 4)
    rng = np.random.default_rng(11)
    for f, g in _random_states(rng, 300):
        f1, g1 = lb.collide(f, g)
        f2, g2 = mr.collide(f, g)
        assert np.abs(f1 - f2).max() <= 1e-15
        assert np.abs(g1 - g2).max() <= 1e-15


def test_lbgk_rates(oracle_mod):
    """One rate per distribution: s_q = s_nu and sigma_e = sigma_nu = sigma_k,
    the viscous and diffusive rates unchanged."""
    O = oracle_mod
    m = O.derive(256, 1e4, 0.01, 0.1)
    b = O.derive(256, 1e4, 0.01, 0.1, collision=O.LBGK)
    assert b["s_nu"] == m["s_nu"] and b["sigma_k"] == m["sigma_k"]
    assert b["s_q"] == b["s_nu"] and b["sigma_e"] == b["sigma_k"] and b["sigma_nu"] == b["sigma_k"]
    assert m["s_q"] != m["s_nu"]


def test_lbgk_equilibria_are_fixed_points(oracle_mod):
    """Without force the textbook equilibria are left unchanged, whatever
    the rates (the MRT moments of Eq. 34 with reading R1 and of Eq. 42)."""
    O = oracle_mod
    o = O.Oracle(32, 1e4, 0.01, collision=O.LBGK, gbeta_override=0.0)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    e = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
    a = o.derived()["a"]
    rng = np.random.default_rng(3)
    for _ in range(50):
        drho, u, v, th = rng.uniform(-0.02, 0.02), *rng.uniform(-0.1, 0.1, 2), rng.uniform(-1, 1)
        eu = e @ np.array([u, v])
        f = w * (drho + 3 * eu + 4.5 * eu ** 2 - 1.5 * (u * u + v * v))
        g = np.array([(1 - a) / 5] + [(4 + a) / 20] * 4) * th + 0.5 * th * (e[:5] @ np.array([u, v]))
        f2, g2 = o.collide(f, g)
        assert np.abs(f2 - f).max() <= 1e-16 and np.abs(g2 - g).max() <= 1e-15


def _tg_rate_lbgk(O, n, nu, U0=1e-6, t1=50, t2=250):
    o = O.Oracle(n, _ra_for(n, nu, 1.0), 1.0, bc=O.PERIODIC, gbeta_override=0.0, collision=O.LBGK)
    k = 2 * np.pi / n
    X, Y = np.meshgrid(np.arange(n), np.arange(n))
    o.set_equilibrium(U=-U0 * np.cos(k * X) * np.sin(k * Y), V=U0 * np.sin(k * X) * np.cos(k * Y))
    o.step(t1)
    a1 = np.sqrt((o.fields()[0] ** 2).sum())
    o.step(t2 - t1)
    a2 = np.sqrt((o.fields()[0] ** 2).sum())
    return -np.log(a2 / a1) / (t2 - t1), 2 * nu * k * k


def test_lbgk_taylor_green_decay(oracle_mod):
    """nu = (1/s_nu - 1/2)/3 holds for LBGK too; the lattice error is O(k^2)."""
    r16, a16 = _tg_rate_lbgk(oracle_mod, 16, 0.05)
    r32, a32 = _tg_rate_lbgk(oracle_mod, 32, 0.05)
    e16, e32 = abs(r16 / a16 - 1), abs(r32 / a32 - 1)
    assert e16 < 0.01 and e32 < 0.0025
    assert 3.0 < e16 / e32 < 5.0


def _thermal_rate_lbgk(O, n, alpha):
    o = O.Oracle(n, _ra_for(n, alpha, 1.0), 1.0, bc=O.PERIODIC, gbeta_override=0.0, collision=O.LBGK)
    k = 2 * np.pi / n
    X, _ = np.meshgrid(np.arange(n), np.arange(n))
    o.set_equilibrium(theta=0.1 * np.sin(k * X))
    o.step(20)
    a1 = np.sqrt((o.fields()[2] ** 2).sum())
    o.step(180)
    a2 = np.sqrt((o.fields()[2] ** 2).sum())
    return -np.log(a2 / a1) / 180, alpha * k * k


def test_lbgk_thermal_decay(oracle_mod):
    """A periodic temperature mode decays at alpha k^2 with sigma_k from
    Eq. 43; the O(k^2) lattice error (larger than with MRT's sigma_e, which
    Eq. 39 ties to sigma_k) drops about fourfold from 16^2 to 32^2."""
    r16, a16 = _thermal_rate_lbgk(oracle_mod, 16, 0.05)
    r32, a32 = _thermal_rate_lbgk(oracle_mod, 32, 0.05)
    e16, e32 = abs(r16 / a16 - 1), abs(r32 / a32 - 1)
    assert e32 < 0.004
    assert 3.0 < e16 / e32 < 5.0


def test_lbgk_cavity_conserves_mass_and_conducts(oracle_mod):
    """In the cavity LBGK conserves mass to round-off and, without buoyancy,
    reaches the exact linear conduction profile with Nu = 1 (Eqs. 44-45 act
    on the populations, whatever the collision operator)."""
    O = oracle_mod
    n = 12
    o = O.Oracle(n, 48.0, 0.01, gbeta_override=0.0, collision=O.LBGK)
    o.set_theta(np.zeros((n, n)))
    m0 = o.get_state()[0].sum()
    o.step(1500)
    assert abs(o.get_state()[0].sum() - m0) < 1e-13
    T = o.fields()[2]
    xc = (np.arange(n) + 0.5) / n
    np.testing.assert_allclose(T, np.broadcast_to(0.5 - xc, (n, n)), atol=1e-12)
    assert abs(o.nusselt(0)[0] - 1.0) < 1e-11


def test_lbgk_and_mrt_steady_nusselt_agree(oracle_mod):
    """Air-like convection where both schemes are stable (Ra 1e4, Pr 0.71,
    24^2): the operators differ (the fields are not identical) but both
    steady hot-wall Nusselt numbers lie within 3 % of the classical
    benchmark value 2.243 for this case (de Vahl Davis, 1983), and of each
    other (2.271 and 2.230 at this coarse grid)."""
    O = oracle_mod
    n = 24
    out = []
    for coll in (O.MRT, O.LBGK):
        o = O.Oracle(n, 1e4, 0.71, collision=coll)
        o.set_theta(np.zeros((n, n)))
        o.step(12000)
        out.append((o.nusselt(0)[0], o.fields()[0]))
    (nu_m, U_m), (nu_b, U_b) = out
    assert np.abs(U_m - U_b).max() > 1e-9
    assert abs(nu_b / nu_m - 1) < 0.03, (nu_m, nu_b)
    assert abs(nu_m / 2.243 - 1) < 0.03 and abs(nu_b / 2.243 - 1) < 0.03
