"""Seeded synthetic inputs for the Jacobi transform workloads.

This module holds only random-number recipes and sizes; it contains none of
the transform's arithmetic.  Both the oracle side and the GPU side receive the
same arrays from here.

The paper measures on random vectors at synthetic sizes with a = b
(Section 4.1, eq. (61); Section 4); there is no dataset to stand in for.
"""
from __future__ import annotations

import numpy as np

# 1D uniform forward, n = 1024, (a, b) = (0.25, -0.35), tol 1e-12, fp64.
C1 = dict(name="1d_n1024", n=(1024,), ab=((0.25, -0.35),), tol=1e-12, seed=101)
# 2D 1024 x 1024, axis 0 (0.25, -0.35), axis 1 (-0.4, 0.1), tol 1e-12.
C2 = dict(name="2d_n1024", n=(1024, 1024), ab=((0.25, -0.35), (-0.4, 0.1)), tol=1e-12, seed=102)
# 3D 256^3, (0.3, 0.3) on every axis, tol 1e-7, decaying spectrum.
C3 = dict(name="3d_n256", n=(256, 256, 256), ab=((0.3, 0.3),) * 3, tol=1e-7, seed=103)


def normal(shape, seed: int) -> np.ndarray:
    """i.i.d. N(0, 1) fp64 of the given shape."""
    return np.random.default_rng(seed).standard_normal(shape)


def decaying(shape, seed: int, power: float = 1.5) -> np.ndarray:
    """z / (1 + i + j + k + ...)^power with z i.i.d. N(0,1); indices are degrees."""
    z = np.random.default_rng(seed).standard_normal(shape)
    deg = np.zeros(shape)
    for axis, n in enumerate(shape):
        sh = [1] * len(shape)
        sh[axis] = n
        deg = deg + np.arange(n, dtype=np.float64).reshape(sh)
    return z / (1.0 + deg) ** power


def config_input(cfg: dict) -> np.ndarray:
    if cfg is C3:
        return decaying(cfg["n"], cfg["seed"])
    return normal(cfg["n"], cfg["seed"])


def random_params(rng: np.random.Generator, d: int, lo: float = -0.5, hi: float = 0.5):
    """(a, b) per axis, i.i.d. uniform in (lo, hi)."""
    return tuple((float(rng.uniform(lo, hi)), float(rng.uniform(lo, hi))) for _ in range(d))


def log_uniform_int(rng: np.random.Generator, lo: int, hi: int) -> int:
    """rint(exp(U(ln lo, ln hi)))."""
    return int(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi)))))


def batch_1d(count: int, seed: int = 104, nmin: int = 64, nmax: int = 16384):
    """Ragged batch of independent 1D transforms: list of (n, (a, b), alpha)."""
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(count):
        n = log_uniform_int(rng, nmin, nmax)
        ab = random_params(rng, 1)[0]
        items.append((n, ab, rng.standard_normal(n)))
    return items


def batch_2d(count: int, seed: int = 1041, nmin: int = 32, nmax: int = 512):
    """Ragged batch of independent 2D transforms: list of ((n0, n1), params, alpha)."""
    rng = np.random.default_rng(seed)
    items = []
    for _ in range(count):
        n = (log_uniform_int(rng, nmin, nmax), log_uniform_int(rng, nmin, nmax))
        items.append((n, random_params(rng, 2), rng.standard_normal(n)))
    return items


def serving_pairs(seed: int = 105, count: int = 16):
    """The (a, b) pairs a serving stream draws from: `count` pairs drawn once,
    each entry uniform in (-0.5, 0.5)."""
    rng = np.random.default_rng(seed)
    return [(float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-0.5, 0.5))) for _ in range(count)]


def serving_stream(count: int, seed: int = 105):
    """Request descriptors of the mixed serving stream: per request
    (d, shape, params, direction) with d = 1, 2, 3 at probabilities
    0.4 / 0.4 / 0.2; each axis's n log-uniform in [64, 4096] (1D), [64, 1024]
    (2D) or [32, 256] (3D); (a, b) per axis from the 16 serving pairs;
    forward or inverse with probability 1/2 each (0 = forward, 1 = inverse).
    Inputs are drawn separately (i.i.d. N(0, 1))."""
    pairs = serving_pairs(seed)
    rng = np.random.default_rng(seed + 1)
    ranges = {1: (64, 4096), 2: (64, 1024), 3: (32, 256)}
    out = []
    for _ in range(count):
        d = int(rng.choice([1, 2, 3], p=[0.4, 0.4, 0.2]))
        lo, hi = ranges[d]
        shape = tuple(log_uniform_int(rng, lo, hi) for _ in range(d))
        params = tuple(pairs[int(rng.integers(0, len(pairs)))] for _ in range(d))
        direction = int(rng.integers(0, 2))
        out.append((d, shape, params, direction))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 106) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
