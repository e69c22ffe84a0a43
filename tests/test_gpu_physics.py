"""The paper's cavity cases on the GPU (Section 4, Table 1) at 256^2,
Ma = 0.1, to Fo = 4: time-averaged hot-wall Nusselt numbers against the
printed values, the trends the paper states, and the FP32 path against the
FP64 path on the oscillation statistics (within 1 %)."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
PAPER = {c["case"]: c for c in GOLDEN["cases"]}


@pytest.fixture(scope="module")
def runs():
    from paper_1601_04633_amd.study import CASES, run_case
    out = {}
    for case in (1, 2, 3, 4):
        Ra, Pr = CASES[case]
        for prec in ("fp32", "fp64"):
            print(f"[physics] case {case} {prec}", flush=True)
            out[(case, prec)] = run_case(256, Ra, Pr, 4.0, 2.0 if case > 1 else 3.0, prec)
    return out


def test_case1_steady_values(runs):
    r = runs[(1, "fp64")]
    p = PAPER[1]
    assert abs(r["mean"] / p["nu_avg"] - 1) < 0.01
    assert abs(r["nu_max"] / p["nu_max"] - 1) < 0.01
    assert abs(r["y_nu_max"] - p["y_nu_max"]) < 0.01


@pytest.mark.parametrize("case", [2, 3])
def test_oscillatory_means(runs, case):
    r = runs[(case, "fp64")]
    assert r["regime"] == "oscillatory"
    assert abs(r["mean"] / PAPER[case]["nu_mean"] - 1) < 0.02


def test_trends_stated_by_the_paper(runs):
    """Lower Pr at fixed Ra: weaker convection, larger oscillation; higher
    Ra at fixed Pr: stronger convection (Conclusions)."""
    m = {c: runs[(c, "fp64")]["mean"] for c in (1, 2, 3, 4)}
    assert m[3] < m[2] and m[1] < m[2] < m[4]
    assert runs[(3, "fp64")]["amplitude"] > runs[(2, "fp64")]["amplitude"]


@pytest.mark.parametrize("case", [2, 3, 4])
def test_fp32_matches_fp64_on_oscillation_statistics(runs, case):
    a, b = runs[(case, "fp32")], runs[(case, "fp64")]
    for key in ("mean", "amplitude", "period_steps"):
        assert abs(a[key] / b[key] - 1) < 0.01, (key, a[key], b[key])


def test_config_256_pr0005_fp32_vs_fp64():
    """256^2, Ra 1e4, Pr 0.005, 200,000 steps in FP32 and FP64: the Nusselt
    series statistics agree within 1 %, the final hot-wall Nu within 1e-4
    and the final U, V, theta fields within 1e-5 (field-norm relative)."""
    from paper_1601_04633_amd import inputs
    from paper_1601_04633_amd.analysis import oscillation_stats
    from paper_1601_04633_amd.dmrt import Cavity
    res = {}
    for prec in ("fp32", "fp64"):
        c = Cavity(n=256, Ra=1e4, Pr=0.005, precision=prec)
        c.set_theta(inputs.theta_noise(256, 1601))
        c.nu_series(10, 20000)
        c.step(200000)
        s = c.nu_series_read()
        st = oscillation_stats(s[10000:], 10, 256, c.derived()["alpha"])
        res[prec] = (st, c.fields(), c.nusselt(0)[0])
    (s32, f32, n32), (s64, f64, n64) = res["fp32"], res["fp64"]
    ferr = {nm: np.linalg.norm(a - b) / np.linalg.norm(b) for nm, a, b in zip("UVT", f32[:3], f64[:3])}
    print(f"[physics] 256^2 Pr 0.005 fp32 vs fp64: mean {abs(s32['mean'] / s64['mean'] - 1):.2e}, "
          f"window p-p {abs(s32['peak_to_peak_window'] / s64['peak_to_peak_window'] - 1):.2e}, "
          f"Nu {abs(n32 / n64 - 1):.2e}, fields {ferr}", flush=True)
    assert abs(s32["mean"] / s64["mean"] - 1) < 0.01
    assert abs(s32["peak_to_peak_window"] / s64["peak_to_peak_window"] - 1) < 0.01
    assert abs(n32 / n64 - 1) < 1e-4
    # measured 1.1e-7 (U), 1.3e-7 (V), 1.8e-7 (theta): the FP32 path's bar
    for nm, e in ferr.items():
        assert e < 1e-5, (nm, e)
