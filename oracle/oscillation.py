"""TEST INFRASTRUCTURE ONLY: statistics of a Nusselt-number time series, as
the paper characterises its oscillatory runs (Section 4, Table 1: mean
Nusselt number, oscillation amplitude and period).

The paper does not define its amplitude or period; the readings used here:
  * the analysed window is cut to whole periods: from the first to the last
    upward crossing of the series' mean (linearly interpolated between
    samples); the mean is taken again over the samples of that window and the
    crossings of the new mean located again;
  * mean      = average of the samples inside the whole-period window;
  * amplitude = half the peak-to-peak range of those samples;
  * period    = (last crossing - first crossing) / (number of crossings - 1),
    in steps (samples x stride).

Written for the oracle side independently of the GPU package's own
post-processing; both sides of a parity test pass their series through this
one function.  Pinned by tests/test_oracle_oscillation.py (sinusoids and
other periodic signals with known mean, amplitude and period).
"""
from __future__ import annotations

import math


def upward_crossings(x, level):
    """Fractional sample positions where the series rises through level:
    x[i] < level <= x[i + 1], at i + (level - x[i]) / (x[i + 1] - x[i])."""
    out = []
    for i in range(len(x) - 1):
        a, b = x[i], x[i + 1]
        if a < level <= b:
            out.append(i + (level - a) / (b - a))
    return out


def stats(series, stride):
    """series: samples every `stride` steps.  Returns a dict with mean,
    amplitude, period_steps and periods (whole periods in the window), or
    regime "not periodic" when fewer than two whole periods are present."""
    x = [float(v) for v in series]
    if not x or not all(math.isfinite(v) for v in x):
        return {"regime": "non-finite or empty"}
    level = sum(x) / len(x)
    for _ in range(2):
        c = upward_crossings(x, level)
        if len(c) < 3:
            return {"regime": "not periodic", "mean": level}
        lo, hi = math.ceil(c[0]), math.floor(c[-1])
        window = x[lo:hi + 1]
        level = sum(window) / len(window)
    c = upward_crossings(x, level)
    lo, hi = math.ceil(c[0]), math.floor(c[-1])
    window = x[lo:hi + 1]
    return {
        "regime": "oscillatory",
        "mean": sum(window) / len(window),
        "amplitude": (max(window) - min(window)) / 2.0,
        "period_steps": (c[-1] - c[0]) / (len(c) - 1) * stride,
        "periods": len(c) - 1,
    }
