"""Pins of the CPU reference gradient (oracle/torch_ref.py, automatic
differentiation of a vectorised FP64 restatement of the oracle) against the
C oracle itself: identical forward, and gradients equal to central
differences of the C oracle's objective (no GPU)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def case():
    from paper_1601_04633_amd import inputs
    n = 16
    return dict(n=n, Ra=1e4, Pr=0.01, tw=inputs.hot_wall_profile(n, 5),
                t0=inputs.theta_noise(n, 6, amp=1e-2), N=200, K=50)


def test_reference_forward_matches_oracle(oracle_mod, case):
    from oracle.torch_ref import Reference
    n = case["n"]
    r = Reference(n, case["Ra"], case["Pr"])
    F = r.fields_after(case["tw"], case["t0"], case["N"])
    o = oracle_mod.Oracle(n, case["Ra"], case["Pr"])
    o.set_hot_wall(case["tw"])
    o.set_theta(case["t0"])
    o.step(case["N"])
    for a, b in zip(F, o.fields()):
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
    with torch.no_grad():
        Jr = float(r.objective(torch.tensor(case["tw"]), torch.tensor(case["t0"]), case["N"],
                               case["K"]))
    o2 = oracle_mod.Oracle(n, case["Ra"], case["Pr"])
    o2.set_hot_wall(case["tw"])
    o2.set_theta(case["t0"])
    Jo = o2.objective(case["N"], case["K"])
    assert abs(Jr - Jo) <= 1e-13 * abs(Jo)


def test_reference_gradient_matches_oracle_finite_differences(case):
    from oracle import fd
    from oracle.torch_ref import Reference
    n = case["n"]
    r = Reference(n, case["Ra"], case["Pr"])
    J, gw, g0 = r.gradient(case["tw"], case["t0"], case["N"], case["K"], segment=50)
    rng = np.random.default_rng(9)
    dirs, expect = [], []
    for y in (0, 5, 11, 15):
        dirs.append((np.eye(n)[y], np.zeros((n, n))))
        expect.append(gw[y])
    for idx in rng.choice(n * n, size=4, replace=False):
        d0 = np.zeros(n * n)
        d0[idx] = 1.0
        dirs.append((np.zeros(n), d0.reshape(n, n)))
        expect.append(g0.reshape(-1)[idx])
    for _ in range(2):
        dw = rng.standard_normal(n)
        d0 = rng.standard_normal((n, n))
        nrm = np.sqrt((dw ** 2).sum() + (d0 ** 2).sum())
        dirs.append((dw / nrm, d0 / nrm))
        expect.append((gw * dw).sum() / nrm + (g0 * d0).sum() / nrm)
    got = fd.directional_derivatives(n, case["Ra"], case["Pr"], case["tw"], case["t0"],
                                     case["N"], case["K"], dirs, h=1e-6, workers=4)
    scale = max(np.abs(gw).max(), np.abs(g0).max())
    for e, g in zip(expect, got):
        assert abs(e - g) <= 1e-6 * max(abs(e), 1e-3 * scale), (e, g)
