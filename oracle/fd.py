"""TEST INFRASTRUCTURE ONLY: central finite differences of the gradient
problem's objective on the FP64 C oracle.

J(theta_w, theta0) = mean hot-wall Nu_avg (Eqs. 18-19) over the last K of N
steps of the cavity started at rest with temperature theta0.  The workers
are plain functions so that a spawn-based process pool can run many oracle
evaluations in parallel on the host cores.
"""
from __future__ import annotations

import numpy as np


def objective(n, Ra, Pr, theta_w, theta0, N, K, Ma=0.1):
    from oracle import oracle as O
    o = O.Oracle(n, Ra, Pr, Ma)
    o.set_hot_wall(np.asarray(theta_w, dtype=np.float64))
    o.set_theta(np.asarray(theta0, dtype=np.float64).reshape(n, n))
    return o.objective(N, K)


def central_difference(args):
    """args = (n, Ra, Pr, theta_w, theta0, N, K, direction_w, direction_0, h):
    (J(x + h d) - J(x - h d)) / (2 h) for the direction d = (d_w, d_0)."""
    n, Ra, Pr, tw, t0, N, K, dw, d0, h = args
    tw = np.asarray(tw, dtype=np.float64)
    t0 = np.asarray(t0, dtype=np.float64)
    jp = objective(n, Ra, Pr, tw + h * dw, t0 + h * d0, N, K)
    jm = objective(n, Ra, Pr, tw - h * dw, t0 - h * d0, N, K)
    return (jp - jm) / (2 * h)


def directional_derivatives(n, Ra, Pr, theta_w, theta0, N, K, directions, h=1e-6, workers=8):
    """directions: list of (d_w (n,), d_0 (n, n)).  Returns the central
    differences, evaluated in a spawn process pool."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(n, Ra, Pr, theta_w, theta0, N, K, np.asarray(dw, dtype=np.float64),
             np.asarray(d0, dtype=np.float64), h) for dw, d0 in directions]
    if workers <= 1:
        return [central_difference(j) for j in jobs]
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(central_difference, jobs))
