"""Runs of the paper's cavity cases (Section 4, Table 1) through the C ABI,
with the Nusselt time series recorded on the device and summarised by
``analysis.oscillation_stats``.

python -m paper_1601_04633_amd.study --case 2 --n 256 --fo 8 --from-fo 4 \
    [--precision fp32] [--Ma 0.1] [--paper-mode] [--stride 10]
prints one JSON line per run.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs
from .analysis import oscillation_stats

# Table 1 of the paper
CASES = {1: (1e4, 0.01), 2: (5e4, 0.01), 3: (5e4, 0.005), 4: (1e5, 0.01)}


def run_case(n, Ra, Pr, fo_total, fo_from, precision="fp32", Ma=0.1, paper_mode=False,
             stride=10, seed=1601, keep_series=False):
    from .dmrt import Cavity, DMRT_Q5_PAPER, DMRT_Q5_FIXED_A
    c = Cavity(n=n, Ra=Ra, Pr=Pr, Ma=Ma, precision=precision,
               q5_mode=DMRT_Q5_PAPER if paper_mode else DMRT_Q5_FIXED_A)
    d = c.derived()
    steps_per_fo = n * n / d["alpha"]
    steps = int(round(fo_total * steps_per_fo))
    c.set_theta(inputs.theta_noise(n, seed))
    c.nu_series(stride, steps // stride + 8)
    t = time.perf_counter()
    c.step(steps)
    series = c.nu_series_read()
    secs = time.perf_counter() - t
    k0 = int(fo_from * steps_per_fo) // stride
    st = oscillation_stats(series[k0:], stride, n, d["alpha"])
    nu, loc = c.nusselt(0)
    nuc, _ = c.nusselt(1)
    y = (np.arange(n) + 0.5) / n
    st.update(n=n, Ra=Ra, Pr=Pr, Ma=Ma, precision=precision, paper_mode=paper_mode,
              a=d["a"], steps=steps, fo_total=fo_total, fo_from=fo_from, seconds=round(secs, 3),
              final_nu_hot=nu, final_nu_cold=nuc, nu_max=float(loc.max()),
              y_nu_max=float(y[int(loc.argmax())]))
    if keep_series:
        st["series"] = series
    c.close()
    return st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", type=int, choices=sorted(CASES), required=True)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--fo", type=float, default=4.0)
    ap.add_argument("--from-fo", type=float, default=2.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--Ma", type=float, default=0.1)
    ap.add_argument("--paper-mode", action="store_true")
    ap.add_argument("--stride", type=int, default=10)
    a = ap.parse_args()
    Ra, Pr = CASES[a.case]
    st = run_case(a.n, Ra, Pr, a.fo, a.from_fo, a.precision, a.Ma, a.paper_mode, a.stride)
    st["case"] = a.case
    print(json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in st.items()}),
          flush=True)


if __name__ == "__main__":
    main()
