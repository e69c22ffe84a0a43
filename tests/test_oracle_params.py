"""Pins of the oracle's parameter map (Eqs. 9, 11-13, 32, 39, 40, 43) by the
defining relations, not by re-typing the derivation (no GPU)."""
import math

import numpy as np
import pytest

CASES = [(64, 1e3, 0.01), (256, 1e4, 0.005), (1024, 1e5, 0.001), (256, 1e4, 0.01),
         (32, 1e4, 0.01), (64, 1e5, 0.001), (512, 1e3, 0.01)]


@pytest.mark.parametrize("n,Ra,Pr", CASES)
def test_dimensionless_groups_eq9(oracle_mod, n, Ra, Pr):
    """The derived lattice nu, alpha, g beta reproduce Ra, Pr and Ma by their
    definitions in Eq. 9 (H = n with halfway walls, c_s^2 = 1/3, dT = 1)."""
    Ma = 0.1
    d = oracle_mod.derive(n, Ra, Pr, Ma)
    H, dT = n, 1.0
    assert d["H"] == H
    assert math.isclose(d["nu"] / d["alpha"], Pr, rel_tol=1e-14)
    assert math.isclose(d["gbeta"] * dT * H ** 3 * Pr / d["nu"] ** 2, Ra, rel_tol=1e-13)
    assert math.isclose(math.sqrt(d["gbeta"] * dT * H) / math.sqrt(1 / 3), Ma, rel_tol=1e-14)
    # Eq. 11 and 13 coefficients
    assert math.isclose(d["nu"] / H, Ma * math.sqrt(Pr / (3 * Ra)), rel_tol=1e-14)
    assert math.isclose(d["alpha"] / H, Ma * math.sqrt(1 / (3 * Ra * Pr)), rel_tol=1e-14)


@pytest.mark.parametrize("n,Ra,Pr", CASES)
def test_relaxation_rates_eq32_eq39_eq43(oracle_mod, n, Ra, Pr):
    """s_nu gives nu = c_s^2 (1/s_nu - 1/2); s_q makes the product of the
    even/odd relaxation parameters 3/16; Eq. 39's product is 1/6; Eq. 43
    gives back alpha; the D2Q5 weights sum to one."""
    d = oracle_mod.derive(n, Ra, Pr, 0.1)
    assert math.isclose((1 / d["s_nu"] - 0.5) / 3, d["nu"], rel_tol=1e-13)
    assert math.isclose((1 / d["s_nu"] - 0.5) * (1 / d["s_q"] - 0.5), 3 / 16, rel_tol=1e-12)
    assert math.isclose((1 / d["sigma_nu"] - 0.5) * (1 / d["sigma_k"] - 0.5), 1 / 6, rel_tol=1e-12)
    assert d["sigma_e"] == d["sigma_nu"]
    assert math.isclose((4 + d["a"]) / 10 * (1 / d["sigma_k"] - 0.5), d["alpha"], rel_tol=1e-13)
    assert math.isclose(d["w0"] + 4 * d["wm"], 1.0, rel_tol=1e-15)
    assert d["a"] == -2 / 3


def test_paper_mode_eq40(oracle_mod):
    """Mode 1 takes Eq. 40 literally and solves Eq. 43 for a; it is accepted
    only where a < 1 (Ma small enough), and Eq. 45's printed constant
    2 sqrt(3) alpha equals (4 + a)/10 there."""
    O = oracle_mod
    # 256^2, Ra 1e4, Pr 0.01: a < 1 needs Ma below about 0.0098
    d = O.derive(256, 1e4, 0.01, 0.009, q5_mode=O.Q5_PAPER)
    assert math.isclose(1 / d["sigma_k"] - 0.5, math.sqrt(3) / 6, rel_tol=1e-14)
    assert math.isclose(1 / d["sigma_nu"] - 0.5, math.sqrt(3) / 3, rel_tol=1e-14)
    assert d["a"] < 1
    assert math.isclose(2 * math.sqrt(3) * d["alpha"], (4 + d["a"]) / 10, rel_tol=1e-13)
    assert math.isclose((4 + d["a"]) / 10 * (1 / d["sigma_k"] - 0.5), d["alpha"], rel_tol=1e-13)


@pytest.mark.parametrize("n,Ra,Pr", CASES)
def test_paper_mode_rejects_every_ma01_config(oracle_mod, n, Ra, Pr):
    """With Ma = 0.1 the literal Eq. 40 forces a = 20 sqrt(3) alpha - 4 > 1,
    which the paper's own stability condition (a < 1) rules out."""
    O = oracle_mod
    with pytest.raises(O.OracleError) as ei:
        O.derive(n, Ra, Pr, 0.1, q5_mode=O.Q5_PAPER)
    assert ei.value.code == O.EUNSTABLE


def test_modes_coincide_where_paper_mode_is_admissible(oracle_mod):
    """Fixed-a mode with the a that mode 1 computes reproduces mode 1."""
    O = oracle_mod
    p = O.derive(256, 1e4, 0.01, 0.005, q5_mode=O.Q5_PAPER)
    f = O.derive(256, 1e4, 0.01, 0.005, q5_mode=O.Q5_FIXED_A, a=p["a"])
    for k in ("sigma_k", "sigma_e", "sigma_nu", "a", "wm"):
        assert math.isclose(p[k], f[k], rel_tol=1e-12), k


@pytest.mark.parametrize("kw,code", [
    (dict(Ma=0.0), "EUNSTABLE"), (dict(Ma=-0.1), "EUNSTABLE"), (dict(Ra=0.0), "EUNSTABLE"),
    (dict(Pr=-1.0), "EUNSTABLE"), (dict(Ra=float("nan")), "EINVAL"),
    (dict(a=1.0), "EUNSTABLE"), (dict(a=-4.0), "EUNSTABLE"), (dict(a=float("inf")), "EINVAL"),
    (dict(n=1), "EINVAL"),
])
def test_invalid_parameters(oracle_mod, kw, code):
    O = oracle_mod
    args = dict(n=64, Ra=1e3, Pr=0.01, Ma=0.1, a=-2 / 3)
    args.update(kw)
    with pytest.raises(O.OracleError) as ei:
        O.derive(args["n"], args["Ra"], args["Pr"], args["Ma"], a=args["a"])
    assert ei.value.code == getattr(O, code)
