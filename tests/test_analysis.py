"""Oscillation statistics on synthetic series with known answers (no GPU)."""
import numpy as np

from paper_1601_04633_amd.analysis import oscillation_stats


def test_sine_period_amplitude_mean():
    stride, P, A, m = 10, 937.0, 0.05, 2.65
    t = np.arange(5000) * stride
    x = m + A * np.sin(2 * np.pi * t / P + 0.3)
    s = oscillation_stats(x, stride, H=256, alpha=0.9)
    assert s["regime"] == "oscillatory"
    assert abs(s["period_steps"] - P) < 1e-3 * P
    assert abs(s["amplitude"] - A) < 2e-3 * A
    assert abs(s["mean"] - m) < 1e-4
    assert abs(s["period_fo"] - P * 0.9 / 256 ** 2) < 1e-3 * P * 0.9 / 256 ** 2
    assert abs(s["period_fft_steps"] - P) < 0.02 * P


def test_steady_series():
    s = oscillation_stats(np.full(100, 1.95), 100, H=64, alpha=1.0)
    assert s["regime"] == "steady" and s["amplitude"] == 0.0
