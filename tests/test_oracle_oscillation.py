"""Pins of the oracle-side oscillation statistics (oracle/oscillation.py)
against signals whose mean, amplitude and period are known in closed form,
and the GPU package's own post-processing (analysis.py) against it."""
import math

import numpy as np
import pytest

from oracle import oscillation


def _sampled(fn, period, stride, count):
    return [fn(2 * math.pi * (k + 1) * stride / period) for k in range(count)]


@pytest.mark.parametrize("period,phase", [(1167.3, 0.0), (766.35, 1.1), (2810.6, 2.9)])
def test_sinusoid(period, phase):
    """m + A sin(t + phase): mean m, amplitude A, the given period."""
    m, A, stride = 2.7676, 1.38e-3, 10
    x = _sampled(lambda t: m + A * math.sin(t + phase), period, stride, 30000)
    st = oscillation.stats(x, stride)
    assert st["regime"] == "oscillatory"
    assert abs(st["period_steps"] / period - 1) < 1e-7
    # the sampled extremes sit within half a sample of the true ones
    h = math.pi * stride / period
    assert A * math.cos(h) <= st["amplitude"] <= A * (1 + 1e-12)
    assert abs(st["mean"] - m) < 1e-4 * A
    # whole periods only: a partial one may be cut at each end
    total = 30000 * stride / period
    assert total - 2 <= st["periods"] <= total


def test_harmonics_do_not_bias_mean_or_period():
    """A skewed periodic wave m + A sin t + B sin(2t + c): mean m and the
    fundamental period; amplitude = half the exact peak-to-peak range."""
    m, A, B, c, period, stride = -0.4, 0.05, 0.02, 0.7, 1540.2, 10
    fn = lambda t: m + A * math.sin(t) + B * math.sin(2 * t + c)
    x = _sampled(fn, period, stride, 40000)
    st = oscillation.stats(x, stride)
    t = np.linspace(0, 2 * np.pi, 200001)
    exact = np.array([fn(v) for v in t])
    half_ptp = (exact.max() - exact.min()) / 2
    assert abs(st["period_steps"] / period - 1) < 1e-6
    assert abs(st["mean"] - m) < 1e-4 * A
    assert abs(st["amplitude"] / half_ptp - 1) < 1e-3


def test_not_periodic():
    x = [1.0 + 1e-3 * k for k in range(500)]
    assert oscillation.stats(x, 10)["regime"] == "not periodic"
    assert oscillation.stats([1.0, float("nan")], 10)["regime"] == "non-finite or empty"


def test_window_is_whole_periods():
    """A partial period at either end must not bias the mean: a square-ish
    wave cut mid-period has the mean of its whole periods."""
    period, stride = 400.0, 10
    fn = lambda t: 1.0 + (0.5 if math.sin(t) > 0 else -0.5) + 0.01 * math.sin(t)
    x = _sampled(fn, period, stride, 40 * 10 + 13)   # 10 periods and a third
    st = oscillation.stats(x, stride)
    assert abs(st["mean"] - 1.0) < 0.5 * 2 / 40      # at most one sample off balance per period
    assert abs(st["period_steps"] / period - 1) < 1e-2


def test_gpu_package_post_processing_agrees():
    """analysis.oscillation_stats (used by study.py) gives the oracle-side
    statistics on the same series."""
    from paper_1601_04633_amd.analysis import oscillation_stats
    m, A, B, period, stride = 2.8, 0.03, 0.004, 2810.6, 10
    x = _sampled(lambda t: m + A * math.sin(t) + B * math.sin(3 * t + 0.2), period, stride, 30000)
    a = oscillation_stats(np.array(x), stride, 128, 1.0)
    b = oscillation.stats(x, stride)
    assert abs(a["period_steps"] / b["period_steps"] - 1) < 1e-9
    assert abs(a["amplitude"] / b["amplitude"] - 1) < 1e-9
    assert abs(a["mean"] / b["mean"] - 1) < 1e-6
