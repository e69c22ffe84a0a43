"""Autotuner for the launch shapes of libdmrt.

Results never depend on the launch shape (the kernels are bitwise
insensitive to it); only the time does.  The tuner times short runs of the
actual workload and keeps the fastest setting, searching one dimension at a
time from a default (coordinate descent, two sweeps).  Winners are cached
in a JSON file keyed by (device architecture, precision, member sizes).

Batch schedule dimensions (dmrt_batch_set_schedule): tile shape, tile
order, workgroups per launch, and cavity groups sized for the 256 MB
last-level cache that run several steps before the next group; steps per
launch with the tile form (dmrt_batch_set_temporal) or the row-marching
form (dmrt_batch_set_temporal_march, entries ("march", K, B)).
Single-cavity dimensions: steps per launch with the tile kernel and its
rows (dmrt_set_temporal) or with the row-marching kernel and its wave rows
per step group (dmrt_set_temporal_march, entries ("march", K, B)), tile
shape and die-aware tile order (dmrt_set_launch).
Adjoint: steps per backward launch and tile rows (dmrt_adjoint_set_temporal).
"""
from __future__ import annotations

import hashlib
import json
import os
import time

CACHE_PATH = os.environ.get("DMRT_AUTOTUNE_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "dmrt_autotune.json"))

MB = 1 << 20

BATCH_SPACE = {
    "temporal": [(4, 16), ("march", 4, 3), ("march", 6, 2), ("march", 4, 4), ("march", 4, 2), (4, 12),
                 (3, 16), (3, 12), (2, 6), (2, 10), (3, 10), (4, 10), (1, 10)],
    "block": [(64, 4), (64, 2), (64, 8), (128, 2), (128, 4), (256, 1), (64, 1)],
    "order": [1, 0, 2],
    "grid_blocks": [0, 4096, 16384],
    # steps per group round: multiples of 12, so that every steps-per-launch
    # choice (1, 2, 3, 4, 6) divides them and no round ends in single steps
    "group": [(0, 60), (96 * MB, 12), (96 * MB, 36), (160 * MB, 24), (160 * MB, 60),
              (224 * MB, 36)],
}
BATCH_DEFAULT = {"temporal": (4, 16), "block": (64, 4), "order": 1, "grid_blocks": 0,
                 "group": (0, 60)}

CAVITY_SPACE = {
    "temporal": [(4, 16), ("march", 4, 3), ("march", 4, 2), ("march", 4, 4), ("march", 6, 2), ("march", 4, 1), (4, 12),
                 (3, 16), (3, 12), (3, 10), (2, 6), (2, 10), (4, 10), (1, 10)],
    "block": [(256, 1), (128, 2), (64, 4), (512, 1), (128, 1), (64, 1), (256, 2)],
    "xcd_remap": [1, 0],
}
CAVITY_DEFAULT = {"temporal": (4, 16), "block": (256, 1), "xcd_remap": 1}


def _arch():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load_cache():
    try:
        with open(CACHE_PATH) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(key, value):
    cache = _load_cache()
    cache[key] = value
    try:
        os.makedirs(os.path.dirname(CACHE_PATH), exist_ok=True)
        tmp = CACHE_PATH + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, CACHE_PATH)
    except OSError:
        pass


def _timer(stream_ptr, sync):
    """Returns (start, stop) closures timing work on the handle's stream:
    HIP events on that stream when its pointer is given, else host time
    with sync() (the handle's own synchronisation) before the stop."""
    try:
        import torch
        ext = torch.cuda.ExternalStream(stream_ptr) if stream_ptr else None
    except Exception:
        ext = None
    if ext is not None:
        import torch
        ev = [torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]

        def start():
            ev[0].record(ext)

        def stop():
            ev[1].record(ext)
            ev[1].synchronize()
            return ev[0].elapsed_time(ev[1]) * 1e-3
        return start, stop
    t = [0.0]

    def start():
        t[0] = time.perf_counter()

    def stop():
        sync()
        return time.perf_counter() - t[0]
    return start, stop


def _coordinate_search(space, default, measure, sweeps=2):
    best = dict(default)
    best_t = measure(best)
    trials = [(dict(best), best_t)]
    for _ in range(sweeps):
        improved = False
        for dim, values in space.items():
            for v in values:
                if v == best[dim]:
                    continue
                cand = dict(best)
                cand[dim] = v
                t = measure(cand)
                trials.append((dict(cand), t))
                if t < best_t:
                    best, best_t, improved = cand, t, True
        if not improved:
            break
    return best, best_t, trials


def batch_key(batch):
    sizes = sorted(batch.n(i) for i in range(batch.count))
    h = hashlib.sha1(json.dumps(sizes).encode()).hexdigest()[:12]
    return f"batch|{_arch()}|{'fp64' if batch.precision == 1 else 'fp32'}|{len(sizes)}|{h}"


def apply_batch(batch, cfg):
    bx, by = cfg["block"]
    gb, gs = cfg["group"]
    batch.set_schedule(block_x=bx, block_y=by, order=cfg["order"],
                       grid_blocks=cfg["grid_blocks"], group_bytes=gb, group_steps=gs)
    t = tuple(cfg.get("temporal", (1, 10)))
    if t[0] == "march":
        batch.set_temporal_march(t[1], t[2], t[3] if len(t) > 3 else 0)
    else:
        batch.set_temporal(*t)


def tune_batch(batch, stream_ptr=None, min_steps=128, use_cache=True, verbose=False):
    """Pick the fastest schedule for this batch; leaves it applied.
    Returns (config, seconds per step, trials)."""
    key = batch_key(batch)
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            cfg = {"temporal": tuple(hit.get("temporal", (1, 10))), "block": tuple(hit["block"]),
                   "order": hit["order"], "grid_blocks": hit["grid_blocks"],
                   "group": tuple(hit["group"])}
            apply_batch(batch, cfg)
            return cfg, hit.get("sec_per_step"), []
    start, stop = _timer(stream_ptr, batch.sync)

    def measure(cfg):
        apply_batch(batch, cfg)
        g = cfg["group"][1]
        steps = max(min_steps, g) // g * g
        batch.step(2 * g)           # builds the captured graph
        batch.sync()
        start()
        batch.step(steps)
        t = stop() / steps
        if verbose:
            print(f"[autotune] batch {cfg} {t * 1e6:.1f} us/step", flush=True)
        return t

    best, best_t, trials = _coordinate_search(BATCH_SPACE, BATCH_DEFAULT, measure)
    apply_batch(batch, best)
    _store_cache(key, {"temporal": list(best["temporal"]), "block": list(best["block"]),
                       "order": best["order"],
                       "grid_blocks": best["grid_blocks"], "group": list(best["group"]),
                       "sec_per_step": best_t})
    return best, best_t, trials


def tune_cavity(cavity, stream_ptr=None, steps=256, use_cache=True, verbose=False):
    """Pick the fastest single-cavity launch shape; leaves it applied."""
    # the search space depends on the wall configuration (K-step forms exist
    # for the cavity only), so it is part of the key
    key = (f"cavity|{_arch()}|{'fp64' if cavity.params.precision == 1 else 'fp32'}|{cavity.n}"
           f"|bc{cavity.params.bc_mode}")
    if cavity.params.bc_mode != 0:
        space = {k: v for k, v in CAVITY_SPACE.items() if k != "temporal"}
        space["temporal"] = [(1, 10)]
    else:
        space = CAVITY_SPACE
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            apply_cavity(cavity, {"temporal": tuple(hit["temporal"]), "block": tuple(hit["block"]),
                                  "xcd_remap": hit["xcd_remap"]})
            return hit, hit.get("sec_per_step"), []
    start, stop = _timer(stream_ptr, cavity.sync)

    def measure(cfg):
        apply_cavity(cavity, cfg)
        cavity.step(128)
        cavity.sync()
        start()
        cavity.step(steps)
        t = stop() / steps
        if verbose:
            print(f"[autotune] cavity n={cavity.n} {cfg} {t * 1e6:.2f} us/step", flush=True)
        return t

    default = dict(CAVITY_DEFAULT)
    default["temporal"] = space["temporal"][0]
    best, best_t, trials = _coordinate_search(space, default, measure, sweeps=1)
    apply_cavity(cavity, best)
    _store_cache(key, {"temporal": list(best["temporal"]), "block": list(best["block"]),
                       "xcd_remap": best["xcd_remap"], "sec_per_step": best_t})
    return best, best_t, trials


ADJOINT_SPACE = [(4, 16), (4, 12), (3, 12), (3, 10), (2, 6), (2, 10), (3, 16), (4, 10), (1, 10)]


def tune_adjoint(cavity, nsteps=2000, avg_last=400, ckpt_every=500, stream_ptr=None, use_cache=True,
                 verbose=False):
    """Pick the fastest steps-per-launch and footprint rows for the backward
    pass of dmrt_adjoint_nu (gradients do not depend on it); leaves it
    applied.  The cavity's theta0 must be set."""
    key = f"adjoint|{_arch()}|{'fp64' if cavity.params.precision == 1 else 'fp32'}|{cavity.n}|{ckpt_every}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            cavity.adjoint_set_temporal(*hit["temporal"])
            return tuple(hit["temporal"]), hit.get("sec_per_step"), []
    start, stop = _timer(stream_ptr, cavity.sync)
    trials = []
    for kr in ADJOINT_SPACE:
        cavity.adjoint_set_temporal(*kr)
        cavity.adjoint_forward(nsteps, avg_last, ckpt_every)
        cavity.adjoint_backward()                 # buffers and captured graphs
        cavity.adjoint_forward(nsteps, avg_last, ckpt_every)
        start()
        cavity.adjoint_backward()
        t = stop() / nsteps
        trials.append((kr, t))
        if verbose:
            print(f"[autotune] adjoint n={cavity.n} backward {kr} {t * 1e6:.2f} us/step", flush=True)
    best, best_t = min(trials, key=lambda e: e[1])
    cavity.adjoint_set_temporal(*best)
    _store_cache(key, {"temporal": list(best), "sec_per_step": best_t})
    return best, best_t, trials


GRAPH_STEPS = 60       # steps per captured graph: a multiple of every K offered (1..4, 6)


def apply_cavity(cavity, cfg):
    """Applies a single-cavity launch configuration (see CAVITY_SPACE)."""
    cavity.set_launch(cfg["block"][0], cfg["block"][1], cfg["xcd_remap"], GRAPH_STEPS)
    t = cfg["temporal"]
    if t[0] == "march":
        cavity.set_temporal_march(int(t[1]), int(t[2]), int(t[3]) if len(t) > 3 else 0)
    else:
        cavity.set_temporal(int(t[0]), int(t[1]))
