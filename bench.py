"""Benchmark of the double-MRT thermal LBM time step on one MI355X.

A "step" is one time step of the whole hot path over one cavity: pull
streaming with the wall conditions, D2Q9 MRT collision with buoyancy, D2Q5
MRT collision and the store (fused; by default one launch advances four
steps through LDS, workgroups marching up chunks of rows).  Default workload:
the 1024 x 1024 cavity, Ra = 1e5, Pr = 0.001, Ma = 0.1, FP32 storage and
arithmetic, seeded noise initial temperature (synthetic; the paper has no
dataset).

Prints ONE JSON line.  value = MLUPS (million node updates per second, one
node update = one D2Q9 + one D2Q5 node advanced one step) with the state
resident in HBM before the timed region starts.

python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extras]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (D2Q9+D2Q5 node updates/s), % HBM roofline; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak (AMD published)
# Vector-instruction issue peak without packed FP32: one wave64 VALU
# instruction per 4 cycles on each of 256 CUs x 4 SIMDs at 2.4 GHz
# (614.4 G wave instructions/s; 78.6 TFLOP/s if every one were an FMA).
VALU_PEAK_GINSTR = 256 * 4 * 2.4 / 4
WORDS_PER_NODE = 28            # 14 populations read + 14 written per node and launch
# Algorithmic arithmetic of a node update: the 100 floating-point
# instructions of the collision (moments, equilibrium distances, force
# image, relaxation and back-transform; streaming is data movement), i.e.
# 100 wave instructions per 64 node updates.
ALG_VALU_PER_NODE = 100
# committed counter summaries, by (kernel, cavity side)
TRAFFIC_FILES = {
    ("step_kernel<float, 0>", 1024): "step_kernel_cavity_1024_fp32_traffic.json",
    ("stepk_kernel<float, 16, 4>", 1024): "stepk_kernel_K4_R16_cavity_1024_fp32_traffic.json",
    ("stepm_kernel<float, 4, 3>", 1024): "stepm_kernel_K4_B3_cavity_1024_fp32_traffic.json",
    ("stepm_kernel<float, 6, 2>", 1024): "stepm_kernel_K6_B2_cavity_1024_fp32_traffic.json",
    ("stepm_kernel<float, 6, 2>", 2048): "stepm_kernel_K6_B2_cavity_2048_fp32_traffic.json",
    ("stepm_kernel<double, 6, 2>", 1024): "stepm_kernel_K6_B2_cavity_1024_fp64_traffic.json",
}
# launch configuration timed by default (the fastest for this workload on
# MI355X): six steps per launch, workgroups of 6 x 2 wavefronts marching
# up chunks of rows (chunk length chosen to keep one launch resident),
# die-aware order, graphs of 240 steps (a multiple of every steps per launch)
DEFAULT_TEMPORAL = ("march", 6, 2, 0)
DEFAULT_LAUNCH = (256, 1, 1, 240)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1601_04633_amd", "csrc", f)
                  for f in ("dmrt_device.hpp",)]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the device code with comments and blank lines removed, so
    that counter summaries stay valid across comment edits only."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def counter_summary(kernel, n):
    """The committed counter summary of this kernel at this cavity side
    (calibrated HBM bytes per launch, VALU instructions per launch), or None
    when it is missing or was taken on a different kernel source."""
    name = TRAFFIC_FILES.get((kernel, n))
    if name is None:
        return None
    try:
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or t.get("kernel") != kernel:
        return None
    return t


def roofline(kernel, esz, n, spl, us_launch, counters):
    """Roofline entry of one kernel launch advancing an n x n cavity by spl
    steps in us_launch microseconds.

    HBM: a launch must read and write every population of every node once,
    whatever spl (the intermediate states of a K-step launch stay on chip):
    28 words x n^2 algorithmic bytes per launch.  ALU: the algorithmic
    instructions of the spl n^2 node updates (ALG_VALU_PER_NODE per node
    update, 64 node updates per wave instruction) against the issue peak,
    with the instructions the launch actually issues (SQ_INSTS_VALU of the
    committed counter summary, which holds while the kernel source is
    unchanged) beside them.  `bound` is instruction issue when the issued
    rate is closer to its peak than the HBM rate is to its own, else HBM;
    the other is reported beside it.  effective_GBs is 28 words per node update (K n^2
    node updates per launch) over the launch time: above the HBM peak for
    K >= 2 because K - 1 of the K steps never leave the chip."""
    t = us_launch * 1e-6
    hbm_bytes = WORDS_PER_NODE * esz * n * n
    hbm = {"achieved": round(hbm_bytes / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(hbm_bytes / t / 1e9 / HBM_PEAK_GBS, 4),
           "algorithmic_bytes_per_launch": hbm_bytes}
    alu = None
    traffic = None
    if counters:
        traffic = counters.get("bytes_per_launch")
        vi = counters.get("valu_instructions_per_launch")
        if vi:
            alg = spl * n * n * ALG_VALU_PER_NODE / 64
            alu = {"achieved": round(alg / t / 1e9, 1), "peak": VALU_PEAK_GINSTR, "unit": "Ginstr/s",
                   "frac": round(alg / t / 1e9 / VALU_PEAK_GINSTR, 4),
                   "algorithmic_instructions_per_launch": round(alg),
                   "issued_Ginstr_s": round(vi / t / 1e9, 1),
                   "issued_frac": round(vi / t / 1e9 / VALU_PEAK_GINSTR, 4),
                   "valu_instructions_per_launch": vi,
                   "valu_busy_frac_counters": counters.get("valu_busy_frac")}
    # the binding resource by the counters: instruction issue when the
    # issued VALU rate is closer to its peak than the HBM rate is to its own
    issue_binds = alu is not None and alu["issued_frac"] > hbm["frac"]
    main, other, bound = (alu, hbm, "alu") if issue_binds else (hbm, alu, "hbm")
    out = {"bound": bound, "achieved": main["achieved"], "peak": main["peak"], "unit": main["unit"],
           "frac": main["frac"], "traffic": traffic, "kernel": kernel,
           "launch_us": round(us_launch, 3), "steps_per_launch": spl,
           "node_updates_per_launch": spl * n * n,
           "effective_GBs": round(WORDS_PER_NODE * esz * spl * n * n / t / 1e9, 1)}
    out["hbm" if bound == "alu" else "alu"] = other
    if bound == "hbm":
        out["algorithmic_bytes_per_launch"] = hbm_bytes
    else:
        for key in ("algorithmic_instructions_per_launch", "issued_Ginstr_s", "issued_frac",
                    "valu_instructions_per_launch", "valu_busy_frac_counters"):
            out[key] = alu[key]
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / hbm_bytes, 4)
    return out


def parse_temporal(text):
    """'K,R' (tile kernel) or 'march,K,B[,chunk]' (row-marching kernel)."""
    parts = text.split(",")
    if parts[0] == "march":
        vals = [int(v) for v in parts[1:]]
        return ("march", vals[0], vals[1], vals[2] if len(vals) > 2 else 0)
    return tuple(int(v) for v in parts)


def steps_per_launch(temporal):
    return temporal[1] if temporal[0] == "march" else temporal[0]


def kernel_name(temporal, esz):
    t = "float" if esz == 4 else "double"
    if temporal[0] == "march":
        return f"stepm_kernel<{t}, {temporal[1]}, {temporal[2]}>"
    if temporal[0] >= 2:
        return f"stepk_kernel<{t}, {temporal[1]}, {temporal[0]}>"
    return f"step_kernel<{t}, 0>"


def apply_temporal(c, temporal):
    """Sets the cavity's steps per launch; returns the rows per workgroup of
    the row-marching kernel (None for the tile kernel)."""
    if temporal[0] == "march":
        return c.set_temporal_march(temporal[1], temporal[2], temporal[3])
    c.set_temporal(*temporal)
    return None


def device_warmup(ms=100.0):
    """Keeps the GPU busy for about `ms` milliseconds with work unrelated to
    the cavity (an elementwise sine over a 16 MB buffer, vector-ALU bound and
    cache resident), so that a short timed region does not start at idle
    clocks; returns the time spent."""
    import torch
    x = torch.rand(4 << 20, device="cuda")
    torch.cuda.synchronize()
    t = time.perf_counter()
    while (time.perf_counter() - t) * 1e3 < ms:
        for _ in range(16):
            torch.sin(x, out=x)
        torch.cuda.synchronize()
    spent = (time.perf_counter() - t) * 1e3
    del x
    return spent


def time_cavity(n, Ra, Pr, precision, steps, warmup, launch=None, seed=1601, temporal=None, info=None,
                nu_stride=0, settle_ms=0.0):
    """Returns (ms total, MLUPS, avg ms per step, Nu) for `steps` steps timed
    with HIP events on the cavity's own stream; info (a dict) receives the
    chunk rows of the row-marching kernel.  nu_stride > 0 records the
    hot-wall Nusselt series every nu_stride steps meanwhile.  settle_ms > 0
    runs device_warmup for that long right before the warm-up steps."""
    import torch
    from paper_1601_04633_amd import inputs
    from paper_1601_04633_amd.dmrt import Cavity
    stream = torch.cuda.Stream()
    c = Cavity(n=n, Ra=Ra, Pr=Pr, precision=precision, stream=stream.cuda_stream)
    if launch:
        c.set_launch(*launch)
    if temporal:
        chunk = apply_temporal(c, temporal)
        if info is not None:
            info["chunk_rows"] = chunk
    c.set_theta(inputs.theta_noise(n, seed))
    if nu_stride:
        c.nu_series(nu_stride, (warmup + steps) // nu_stride + 8)
    if settle_ms > 0:
        spent = device_warmup(settle_ms)
        if info is not None:
            info["device_warmup_ms"] = round(spent, 1)
    c.step(warmup)
    c.sync()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    c.step(steps)
    t1.record(stream)
    t1.synchronize()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    nu = c.nusselt(0)[0]
    c.close()
    mlups = n * n * steps / (ms * 1e-3) / 1e6
    return ms, mlups, ms / steps, nu


def bench_batch(steps, single_steps, count=64, seed=4633, tune=True):
    """The Ra x Pr sweep (count cavities, sides {64..512}, FP32) in one launch
    per step, against the same cavities stepped one by one with the
    single-cavity kernel (graphs and tuned launch shapes in both)."""
    import torch
    from paper_1601_04633_amd import autotune, inputs
    from paper_1601_04633_amd.dmrt import Batch, Cavity
    specs = inputs.batch_cavities(count, seed)
    members = [dict(n=s, Ra=ra, Pr=pr) for s, ra, pr in specs]
    nodes = sum(m["n"] ** 2 for m in members)
    stream = torch.cuda.Stream()
    b = Batch(members, precision="fp32", stream=stream.cuda_stream)
    for i, m in enumerate(members):
        b.set_theta(i, inputs.theta_noise(m["n"], seed + i))
    cfg = None
    if tune:
        cfg, _, trials = autotune.tune_batch(b, stream_ptr=stream.cuda_stream, use_cache=False)
        log(f"batch: tuned schedule {cfg} after {len(trials)} trials")
    g = cfg["group"][1] if cfg else 64
    steps = max(steps // g, 1) * g
    b.step(2 * g)
    b.sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    b.step(steps)
    t1.record(stream)
    t1.synchronize()
    sec = t0.elapsed_time(t1) * 1e-3
    nu = b.nusselt()
    status = b.status()
    b.close()
    batch_mlups = nodes * steps / sec / 1e6

    # one by one: every member alone for single_steps steps
    total = 0.0
    tuned = {}
    for i, m in enumerate(members):
        c = Cavity(precision="fp32", stream=stream.cuda_stream, **m)
        c.set_theta(inputs.theta_noise(m["n"], seed + i))
        if m["n"] not in tuned:
            tuned[m["n"]] = autotune.tune_cavity(c, stream_ptr=stream.cuda_stream, use_cache=False)[0]
        else:
            autotune.apply_cavity(c, tuned[m["n"]])
        c.step(128)
        c.sync()
        t0.record(stream)
        c.step(single_steps)
        t1.record(stream)
        t1.synchronize()
        total += t0.elapsed_time(t1) * 1e-3
        c.close()
    single_mlups = nodes * single_steps / total / 1e6
    return {"cavities": count, "nodes": nodes, "precision": "fp32",
            "batch_steps_timed": steps, "single_steps_timed_each": single_steps,
            "batch_mlups": round(batch_mlups, 1), "one_by_one_mlups": round(single_mlups, 1),
            "batch_over_one_by_one": round(batch_mlups / single_mlups, 3),
            "roofline": batch_roofline(batch_mlups, cfg),
            "schedule": {k: list(v) if isinstance(v, tuple) else v for k, v in cfg.items()} if cfg else None,
            "single_launch_by_side": {str(k): {"block": list(v["block"]), "xcd_remap": v["xcd_remap"],
                                               "steps_per_launch_rows": list(v["temporal"])}
                                      for k, v in tuned.items()},
            "dead_members": int((status != 0).sum()),
            "nu_hot_wall_mean": float(nu[np.isfinite(nu)].mean())}


def batch_roofline(mlups, cfg):
    """The batched launches move every population of every member once per
    launch: 28 words x 4 B per node per launch, i.e. 112 / K B per node
    update with K steps per launch."""
    t = tuple(cfg["temporal"]) if cfg else (1, 10)
    if t[0] == "march":
        K = int(t[1])
        kernel = f"batch_stepm_kernel<float, {K}, {int(t[2])}>"
    else:
        K = int(t[0])
        kernel = f"batch_stepk_kernel<float, {t[1]}, {K}>" if K >= 2 else "batch_step_kernel<float>"
    gbs = mlups * 1e6 * WORDS_PER_NODE * 4 / K / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": kernel,
            "bytes_per_node_update": WORDS_PER_NODE * 4 / K, "steps_per_launch": K,
            "effective_GBs": round(mlups * 1e6 * WORDS_PER_NODE * 4 / 1e9, 1)}


def adjoint_words(K):
    """Words moved per adjoint step and node at K adjoint steps per launch:
    mu is read and written once per launch (28 / K), the linearisation
    point (u, v, theta) of each step is read once (3); the fused recompute
    of the older segment reads its input state and writes its output state
    once per launch (28 / K) and stores the point of every step (3):
    6 + 56 / K words (K = 1 is the single-step form)."""
    return 6 + 56 / K


def adjoint_roofline(n, t_bwd_step, K, esz=4):
    """Backward pass at K adjoint steps per launch against HBM, with the
    algorithmic words of adjoint_words(K) per adjoint step and node."""
    words = adjoint_words(K)
    gbs = words * esz * n * n / t_bwd_step / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"adjk_fused_kernel<float, R, {K}>" if K >= 2 else "adj_fused_kernel<float>",
            "bytes_per_adjoint_node_update": round(words * esz, 2), "steps_per_launch": K}


def bench_adjoint(n=256, Ra=1e4, Pr=0.01, N=10000, K=2000, C=500, precision="fp32"):
    """Gradient of the mean hot-wall Nu over the last K of N steps (256^2,
    FP32, checkpoints every C): time per step of the plain forward, of the
    checkpointed forward that also accumulates J, and of the backward
    (segment recompute + adjoint kernel), each in its fastest launch
    configuration."""
    import torch
    from paper_1601_04633_amd import autotune, inputs
    from paper_1601_04633_amd.dmrt import Cavity
    stream = torch.cuda.Stream()
    c = Cavity(n=n, Ra=Ra, Pr=Pr, precision=precision, stream=stream.cuda_stream)
    tw = inputs.hot_wall_profile(n, 4633)
    t0 = inputs.theta_noise(n, 1601)
    c.set_hot_wall(tw)
    c.set_theta(t0)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        torch.cuda.synchronize()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        e1.synchronize()
        return out, e0.elapsed_time(e1) * 1e-3

    # the forward reference is the fastest plain stepping of this cavity
    best, _, _ = autotune.tune_cavity(c, stream_ptr=stream.cuda_stream, use_cache=False)
    c.set_theta(t0)
    bwd, _, bwd_trials = autotune.tune_adjoint(c, ckpt_every=C, stream_ptr=stream.cuda_stream,
                                               use_cache=False)
    c.set_theta(t0)
    c.step(1000)                                  # warm-up, graphs
    c.sync()
    _, t_plain = timed(lambda: c.step(N))
    c.adjoint_forward(N, K, C)                     # warm-up: buffers and graphs
    c.adjoint_backward()
    J, t_fwd = timed(lambda: c.adjoint_forward(N, K, C))
    (gw, g0), t_bwd = timed(lambda: c.adjoint_backward())
    c.close()
    return {"workload": f"{n}x{n} cavity, Ra={Ra:g}, Pr={Pr:g}, {precision.upper()}, {N} steps, "
                        f"J = mean hot-wall Nu over the last {K}, checkpoint every {C}",
            "forward_launch": {"block": list(best["block"]), "xcd_remap": best["xcd_remap"],
                               "steps_per_launch_rows": list(best["temporal"])},
            "forward_us_per_step": round(t_plain / N * 1e6, 3),
            "checkpointed_forward_us_per_step": round(t_fwd / N * 1e6, 3),
            "backward_launch": {"steps_per_launch_rows": list(bwd),
                                "tuning_us_per_step": {f"K{k}R{r}": round(t * 1e6, 3)
                                                       for (k, r), t in bwd_trials}},
            "backward_us_per_step": round(t_bwd / N * 1e6, 3),
            "backward_over_forward": round(t_bwd / t_plain, 3),
            "forward_plus_backward_over_forward": round((t_fwd + t_bwd) / t_plain, 3),
            "backward_over_forward_bytes": round(adjoint_words(int(bwd[0]))
                                                 / (28 / steps_per_launch(tuple(best["temporal"]))), 3),
            "roofline": adjoint_roofline(n, t_bwd / N, int(bwd[0]), 8 if precision == "fp64" else 4),
            "J": J, "grad_theta_w_norm": float(np.linalg.norm(gw)),
            "grad_theta0_norm": float(np.linalg.norm(g0))}


def cpu_baseline(n, Ra, Pr, budget_s=15.0):
    """The FP64 oracle on the host (single thread) over a bounded sample of
    the same workload: whole steps of the same cavity until ~budget_s."""
    from oracle import oracle as orc
    from paper_1601_04633_amd import inputs
    o = orc.Oracle(n, Ra, Pr)
    o.set_theta(inputs.theta_noise(n, 1601))
    t = time.perf_counter()
    o.step(1)
    one = time.perf_counter() - t
    k = max(1, int(budget_s / max(one, 1e-9)) - 1)
    t = time.perf_counter()
    o.step(k)
    el = time.perf_counter() - t
    return {"value": round(n * n * k / el / 1e6, 4), "unit": "MLUPS", "cores": 1,
            "kind": "oracle",
            "sample": f"{k} steps of the {n}x{n} cavity (Ra={Ra:g}, Pr={Pr:g}, FP64, "
                      f"single thread), {el:.1f} s"}


def cpu_baseline_all_cores(n, Ra, Pr, rate_1core, budget_s=10.0, max_threads=16):
    """The same oracle, unchanged, on every host core available: one cavity
    per thread, all stepping at once (the C oracle runs with Python's lock
    released, and each handle owns its state), whole-job node updates over
    wall time.  rate_1core (MLUPS) sizes the sample."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as orc
    from paper_1601_04633_amd import inputs
    threads = max(1, min(len(os.sched_getaffinity(0)), max_threads))
    th0 = inputs.theta_noise(n, 1601)
    cavities = []
    for _ in range(threads):
        o = orc.Oracle(n, Ra, Pr)
        o.set_theta(th0)
        cavities.append(o)
    k = max(1, int(budget_s * rate_1core * 1e6 / (n * n)))
    t = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        list(pool.map(lambda o: o.step(k), cavities))
    el = time.perf_counter() - t
    del cavities
    return {"value": round(threads * n * n * k / el / 1e6, 4), "unit": "MLUPS", "cores": threads,
            "kind": "oracle, one cavity per thread",
            "sample": f"{threads} threads x {k} steps of the {n}x{n} cavity (Ra={Ra:g}, Pr={Pr:g}, FP64), "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--Ra", type=float, default=1e5)
    ap.add_argument("--Pr", type=float, default=0.001)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--device-warmup-ms", type=float, default=100.0,
                    help="untimed device work (not cavity steps) before the warm-up steps of the main timing")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--launch", default="", help="block_x,block_y,xcd_remap,graph_steps")
    ap.add_argument("--temporal", default="",
                    help="steps_per_launch,tile_rows or march,steps_per_launch,group_rows[,chunk_rows] "
                         "(default march,4,3)")
    ap.add_argument("--sections", default="main,extras,batch,adjoint,cpu",
                    help="comma list of main, extras, batch, adjoint, cpu")
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--single-steps", type=int, default=2000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library steps a cavity on one GPU "
              "(sharding across GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None

    n, Ra, Pr, prec = args.n, args.Ra, args.Pr, args.precision
    temporal = parse_temporal(args.temporal) if args.temporal else DEFAULT_TEMPORAL
    if launch is None:
        launch = DEFAULT_LAUNCH
    log(f"main: {n}^2 Ra={Ra:g} Pr={Pr:g} {prec} steps={args.steps} warmup={args.warmup} "
        f"launch={launch} temporal={temporal}")
    info = {}
    ms, mlups, ms_step, nu = time_cavity(n, Ra, Pr, prec, args.steps, args.warmup, launch,
                                         temporal=temporal, info=info, settle_ms=args.device_warmup_ms)
    esz = 8 if prec == "fp64" else 4
    spl = steps_per_launch(temporal)        # node updates per node per launch
    us_launch = ms_step * spl * 1e3
    kname = kernel_name(temporal, esz)
    roof = roofline(kname, esz, n, spl, us_launch, counter_summary(kname, n))
    log(f"main: {mlups:.1f} MLUPS, {us_launch:.2f} us/launch, roofline {roof['bound']} "
        f"{roof['achieved']} {roof['unit']} = {roof['frac']:.3f} of peak "
        f"(effective {roof['effective_GBs']} GB/s at 112 B per node update), Nu {nu:.5f}")

    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic: seeded uniform noise of amplitude 1e-4 on theta at rest (numpy PCG64, seed 1601)",
        "config": {"workload": f"differentially heated cavity {n}x{n}, Ra={Ra:g}, Pr={Pr:g}, "
                               f"Ma=0.1, walls +-0.5, {prec.upper()} fused collide-stream step, "
                               f"{spl} step(s) per launch",
                   "global_batch": 1, "nodes": n * n, "parallelism": "single GPU"},
        "roofline": roof,
        "launch": {"block": list(launch[:2]), "xcd_remap": launch[2], "graph_steps": launch[3],
                   "steps_per_launch": spl,
                   **({"kernel": "row-marching", "group_rows": temporal[2],
                       "chunk_rows": info.get("chunk_rows")} if temporal[0] == "march"
                      else {"kernel": "tile", "tile_rows": temporal[1]})},
        "nu_hot_wall": nu,
        # untimed: elementwise work on the device right before the warm-up
        # steps (clocks at their working level for a short timed region)
        "device_warmup_ms": info.get("device_warmup_ms", 0.0),
    }

    if args.calib_copy:
        # a plain copy of known size, 1 GiB read + 1 GiB written per launch
        # (larger than the last-level cache), repeated, so that HBM byte
        # counters can be scaled against the true traffic
        src = torch.ones(256 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(8):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes_each_way"] = src.numel() * 4
        del src, dst
        log("calibration copy: 8 x 1 GiB")

    sections = set(args.sections.split(","))
    if args.no_extras:
        sections -= {"extras", "batch", "adjoint"}
    if args.no_cpu:
        sections -= {"cpu"}

    if "extras" in sections:
        extras = {}
        def extra(name, n_, prec_, steps_, warm_, temporal_):
            _, m, ms_step_, _ = time_cavity(n_, Ra, Pr, prec_, steps_, warm_, launch, temporal=temporal_)
            e = 8 if prec_ == "fp64" else 4
            k = steps_per_launch(temporal_)
            kn = kernel_name(temporal_, e)
            extras[name] = {"mlups": round(m, 1),
                            "roofline": roofline(kn, e, n_, k, ms_step_ * k * 1e3, counter_summary(kn, n_))}

        log("extra: fp32 row-marching with four steps per launch (4 x 3 wavefronts)")
        extra("fp32_march_K4_B3", n, prec, max(args.steps // 5, 2000), 500, ("march", 4, 3, 0))
        log("extra: fp64 same cavity, row-marching (6 steps, 6 x 2 wavefronts) and tile (4 steps, 16 rows)")
        extra("fp64_march_K6_B2", n, "fp64", max(args.steps // 10, 1200), 600, ("march", 6, 2, 0))
        extra("fp64_tile_K4_R16", n, "fp64", max(args.steps // 10, 1200), 600, (4, 16))
        log("extra: fp32 tile kernel (4 steps, 16 rows) and single steps")
        extra("fp32_tile_K4_R16", n, prec, max(args.steps // 5, 2000), 500, (4, 16))
        extra("fp32_single_step", n, prec, max(args.steps // 5, 2000), 500, (1, 10))
        log("extra: the benchmark's launch with the Nusselt series recorded every 10 steps")
        _, mnu, _, _ = time_cavity(n, Ra, Pr, prec, max(args.steps // 5, 2000), 500, launch,
                                   temporal=temporal, nu_stride=10)
        extras["nu_series_stride10_mlups"] = round(mnu, 1)
        log("extra: 2048^2 fp32 control (state larger than the 256 MB last-level cache)")
        extra("fp32_2048_march_K6_B2", 2048, "fp32", 4800, 600, ("march", 6, 2, 0))
        extra("fp32_2048_tile_K4_R16", 2048, "fp32", 4800, 600, (4, 16))
        out["extras"] = extras
    if "batch" in sections:
        log("batch: 64-cavity Ra x Pr sweep vs one by one")
        out["batch"] = bench_batch(args.batch_steps, args.single_steps)
        log(f"batch: {out['batch']['batch_mlups']} MLUPS vs one by one "
            f"{out['batch']['one_by_one_mlups']} MLUPS")

    if "adjoint" in sections:
        log("adjoint: 256^2 FP32 gradient of the mean hot-wall Nu")
        out["adjoint"] = bench_adjoint()
        log(f"adjoint: backward/forward {out['adjoint']['backward_over_forward']}")

    if "cpu" in sections:
        log("cpu baseline (oracle, single thread)")
        out["cpu_baseline"] = cpu_baseline(n, Ra, Pr)
        log("cpu baseline (oracle, every host core)")
        out["cpu_baseline_all_cores"] = cpu_baseline_all_cores(n, Ra, Pr, out["cpu_baseline"]["value"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
