"""Runs of the paper's cavity cases (Section 4, Table 1) through the C ABI,
with the Nusselt time series recorded on the device and summarised by
``analysis.oscillation_stats``.

python -m paper_1601_04633_amd.study --case 2 --n 256 --fo 8 --from-fo 4 \
    [--precision fp32] [--Ma 0.1] [--paper-mode] [--stride 10]
prints one JSON line per run;
python -m paper_1601_04633_amd.study --stability [--n 256] [--steps 100000]
prints the double MRT / double LBGK stability map.
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
    # four steps per launch (bitwise the same states; a Nu sample due inside
    # a launch is taken by that launch)
    if n >= 1024:
        c.set_temporal_march(4, 3, 0)
    else:
        c.set_temporal(4, 16 if n >= 512 else 12)
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


def stability_map(n=256, Ra=(1e3, 1e4, 1e5, 1e6), Pr=(0.001, 0.005, 0.01, 0.05, 0.71),
                  steps=100000, precision="fp32", Ma=0.1, seed=1601, u_runaway=0.5,
                  collisions=("mrt", "lbgk"), temporal=(4, 16), chunks=20):
    """Double MRT against double LBGK over an (Ra, Pr) grid at one
    resolution, all runs in one batched sweep: a member is "nonfinite" when
    its state holds NaN/Inf after ``steps`` steps, "runaway" when a velocity
    exceeds ``u_runaway`` (lattice units; the characteristic velocity is
    Ma/sqrt(3)), else "stable" with its hot-wall Nusselt number.  Points
    whose relaxation rates fall outside (0, 2) are reported as "rejected".
    The state is checked every steps/chunks steps; a non-finite member
    records the first check that found it so."""
    from .dmrt import Batch, DmrtError, derive, make_params
    members, meta, out = [], [], []
    for ra in Ra:
        for pr in Pr:
            for coll in collisions:
                kw = dict(n=n, Ra=ra, Pr=pr, Ma=Ma, collision=coll)
                try:
                    d = derive(make_params(precision=precision, **kw))
                except DmrtError:
                    out.append(dict(Ra=ra, Pr=pr, collision=coll, status="rejected"))
                    continue
                members.append(kw)
                meta.append(dict(Ra=ra, Pr=pr, collision=coll, s_nu=d["s_nu"], s_q=d["s_q"],
                                 sigma_k=d["sigma_k"], sigma_e=d["sigma_e"]))
    b = Batch(members, precision=precision)
    b.set_temporal(*temporal)
    for i in range(len(members)):
        b.set_theta(i, inputs.theta_noise(n, seed))
    t = time.perf_counter()
    died = [None] * len(members)
    chunk = max(1, steps // chunks)
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        b.step(k)
        done += k
        status = b.status()
        for i in range(len(members)):
            if status[i] != 0 and died[i] is None:
                died[i] = done
    secs = time.perf_counter() - t
    nu = b.nusselt()
    for i, m in enumerate(meta):
        rec = dict(m, steps=steps, n=n, precision=precision)
        if status[i] != 0:
            rec["status"] = "nonfinite"
            rec["nonfinite_by_step"] = died[i]
        else:
            U, V, _, _ = b.fields(i)
            umax = float(max(np.abs(U).max(), np.abs(V).max()))
            rec["u_max"] = umax
            rec["status"] = "runaway" if umax > u_runaway else "stable"
            rec["nu_hot"] = float(nu[i])
        out.append(rec)
    b.close()
    return out, secs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", type=int, choices=sorted(CASES))
    ap.add_argument("--stability", action="store_true",
                    help="double MRT vs double LBGK stability map instead of a case")
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--fo", type=float, default=4.0)
    ap.add_argument("--from-fo", type=float, default=2.0)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--Ma", type=float, default=0.1)
    ap.add_argument("--paper-mode", action="store_true")
    ap.add_argument("--stride", type=int, default=10)
    a = ap.parse_args()
    if a.stability:
        recs, secs = stability_map(n=a.n, steps=a.steps, precision=a.precision, Ma=a.Ma)
        for r in recs:
            print(json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}),
                  flush=True)
        print(json.dumps({"sweep_seconds": round(secs, 3)}), flush=True)
        return
    if a.case is None:
        ap.error("--case or --stability is required")
    Ra, Pr = CASES[a.case]
    st = run_case(a.n, Ra, Pr, a.fo, a.from_fo, a.precision, a.Ma, a.paper_mode, a.stride)
    st["case"] = a.case
    print(json.dumps({k: (round(v, 6) if isinstance(v, float) else v) for k, v in st.items()}),
          flush=True)


if __name__ == "__main__":
    main()
