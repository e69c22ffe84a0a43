"""Seeded synthetic inputs shared by the GPU path's callers and the tests.

This module holds random-number recipes only and none of the method's
arithmetic.  Every generator uses numpy's PCG64 bit generator with an explicit
seed, so the same call gives the same bytes on every machine.

The paper (Section 2) fixes the problem but not its initial condition; the
inputs here are the stand-ins: fluid at rest, temperature zero (the midpoint
of the wall temperatures) plus uniform noise, and for the gradient problem a
hot-wall profile perturbed around its nominal value.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def theta_noise(n: int, seed: int, amp: float = 1e-4, base: float = 0.0) -> np.ndarray:
    """(n, n) float64, indexed [y, x]: base + U[-amp, amp) i.i.d. per node."""
    return base + _rng(seed).uniform(-amp, amp, size=(n, n))


def hot_wall_profile(n: int, seed: int, base: float = 0.5, amp: float = 1e-2) -> np.ndarray:
    """(n,) float64 hot-wall temperature per row: base + U[-amp, amp)."""
    return base + _rng(seed).uniform(-amp, amp, size=n)


def batch_cavities(count: int = 64, seed: int = 4633,
                   sides=(64, 128, 256, 512), ra_range=(1e3, 1e5),
                   prs=(0.001, 0.005, 0.01)):
    """Ra x Pr sweep members: list of (side, Ra, Pr).

    side uniform over ``sides``, Ra log-uniform over ``ra_range``, Pr uniform
    over ``prs``; one draw of each per cavity, in that order.
    """
    r = _rng(seed)
    lo, hi = np.log10(ra_range[0]), np.log10(ra_range[1])
    out = []
    for _ in range(count):
        side = int(sides[int(r.integers(0, len(sides)))])
        ra = float(10.0 ** r.uniform(lo, hi))
        pr = float(prs[int(r.integers(0, len(prs)))])
        out.append((side, ra, pr))
    return out


def random_directions(shape, count: int, seed: int) -> np.ndarray:
    """count unit-norm float64 directions of the given shape."""
    r = _rng(seed)
    d = r.standard_normal(size=(count,) + tuple(shape))
    norms = np.sqrt((d.reshape(count, -1) ** 2).sum(axis=1))
    return d / norms.reshape((count,) + (1,) * len(shape))
