"""Statistics of a Nusselt-number time series (host-side post-processing).

The paper characterises its runs by the time-averaged Nusselt number and,
for oscillatory ones, by the oscillation amplitude and period (Section 4).
Here: mean over the analysed window; amplitude = half the peak-to-peak
range over the whole periods in the window (also reported as peak-to-peak);
period = mean spacing of the upward crossings of the mean, linearly
interpolated, cross-checked against the dominant FFT frequency.  Times are
reported in steps, in the convective time tau = steps / H (Eq. 9 with
c = 1) and in the Fourier number Fo = steps * alpha / H^2 (Eq. 20).
"""
from __future__ import annotations

import numpy as np


def crossings_up(x, level):
    """Fractional sample positions where x rises through level."""
    d = x - level
    idx = np.nonzero((d[:-1] < 0) & (d[1:] >= 0))[0]
    frac = -d[idx] / (d[idx + 1] - d[idx])
    return idx + frac


def oscillation_stats(series, stride, H, alpha, steady_rtol=1e-6):
    """series: Nu samples every `stride` steps (already cut to the analysed
    window).  Returns a dict with regime, mean, amplitude, period."""
    x = np.asarray(series, dtype=np.float64)
    mean = float(x.mean())
    out = {"mean": mean, "samples": int(x.size), "stride_steps": int(stride)}
    ptp = float(x.max() - x.min())
    out["peak_to_peak_window"] = ptp
    if ptp <= steady_rtol * abs(mean):
        out.update(regime="steady", amplitude=0.0, period_steps=None, period_tau=None,
                   period_fo=None)
        return out
    c = crossings_up(x, mean)
    if c.size < 3:
        out.update(regime="transient or slow drift", amplitude=ptp / 2, period_steps=None,
                   period_tau=None, period_fo=None)
        return out
    # whole periods between the first and last upward crossing; the mean is
    # re-taken over them (a partial period biases it) and the crossings of
    # that mean located again
    a, b = int(np.ceil(c[0])), int(np.floor(c[-1]))
    mean = float(x[a:b].mean())
    c = crossings_up(x, mean)
    a, b = int(np.ceil(c[0])), int(np.floor(c[-1]))
    seg = x[a:b + 1]
    mean = float(x[a:b].mean())
    out["mean"] = mean
    per_samples = float(np.diff(c).mean())
    per_steps = per_samples * stride
    # FFT cross-check on the mean-removed window
    spec = np.abs(np.fft.rfft(x - mean))
    freqs = np.fft.rfftfreq(x.size, d=stride)
    k = int(np.argmax(spec[1:])) + 1
    out.update(regime="oscillatory", amplitude=float((seg.max() - seg.min()) / 2),
               peak_to_peak=float(seg.max() - seg.min()),
               period_steps=per_steps, period_tau=per_steps / H, period_fo=per_steps * alpha / H ** 2,
               period_fft_steps=float(1.0 / freqs[k]) if freqs[k] > 0 else None,
               periods_in_window=int(c.size - 1),
               period_spread=float(np.diff(c).std() / np.diff(c).mean()))
    return out
