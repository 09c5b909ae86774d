"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only *draws* inputs: grid samples of densities, contrasts,
incident fields and the parameters of discontinuous densities.  It holds no
step of the convolution method itself (no moments, no transforms, no
smoothing), so that the oracle and the GPU path can both consume the same data
without sharing any of the arithmetic that is being checked.

Conventions
-----------
* Grid: ``x_j = j / n`` for ``j`` in ``[0, n)^2`` on the unit square ``D``
  (Section 2.1: the grid G_n includes x = 0 and excludes x = 1).
* Arrays are indexed ``[j1, j2]``; the first index is the x1 coordinate and
  ``j2`` is contiguous in memory.
* All values are generated in float64 with ``numpy.random.default_rng(seed)``
  (PCG64), drawing in the order stated in each function.
"""
from __future__ import annotations

import math

import numpy as np

CENTRE = (0.5, 0.5)
CUT_RADIUS = 0.4


def grid(n: int):
    """Return the coordinate arrays (x1, x2) of the grid j/n, shape (n, n)."""
    t = np.arange(n, dtype=np.float64) / n
    return np.meshgrid(t, t, indexing="ij")


def radius(n: int, centre=CENTRE):
    x1, x2 = grid(n)
    return np.hypot(x1 - centre[0], x2 - centre[1])


def cutoff(n: int, rho: float = CUT_RADIUS) -> np.ndarray:
    """Compactly supported C-infinity bump exp(1 - 1/(1 - r^2/rho^2)) about (0.5, 0.5).

    Evaluated for r < rho only and set to 0 elsewhere (the expression is 0/0 at
    r = rho; it underflows cleanly to 0 just inside).
    """
    r = radius(n)
    out = np.zeros((n, n))
    inside = r < rho
    s = 1.0 - (r[inside] / rho) ** 2
    with np.errstate(over="ignore", under="ignore"):
        out[inside] = np.exp(1.0 - 1.0 / s)
    return out


def bump_density(n: int) -> np.ndarray:
    """Single bump used for the one-apply FP64 case (the cutoff itself)."""
    return cutoff(n)


def gaussian_density(n: int, sigma: float = 0.05) -> np.ndarray:
    """(1/(2 pi sigma^2)) exp(-|y - c|^2 / (2 sigma^2)) about the centre c of D: the
    density of the paper's first convergence example (Section 3.1), sigma = 0.05."""
    r = radius(n)
    return np.exp(-r * r / (2.0 * sigma * sigma)) / (2.0 * np.pi * sigma * sigma)


def smooth_density(n: int, seed: int) -> np.ndarray:
    """Sum of 1..8 Gaussian bumps times the cutoff.

    Draw order (one generator per density): m ~ U{1..8}; then for each bump
    in turn: centre c ~ U[0.3, 0.7]^2 (c1 then c2), width w ~ U[0.03, 0.1]
    (standard deviation), amplitude A ~ N(0, 1).
    u = cut * sum_i A_i exp(-|x - c_i|^2 / (2 w_i^2)).
    """
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 9))
    params = []
    for _ in range(m):
        c1 = rng.uniform(0.3, 0.7)
        c2 = rng.uniform(0.3, 0.7)
        w = rng.uniform(0.03, 0.1)
        a = rng.normal()
        params.append((c1, c2, w, a))
    x1, x2 = grid(n)
    acc = np.zeros((n, n))
    for c1, c2, w, a in params:
        acc += a * np.exp(-((x1 - c1) ** 2 + (x2 - c2) ** 2) / (2.0 * w * w))
    return acc * cutoff(n)


def full_support_density(n: int, seed: int, power: int = 3) -> np.ndarray:
    """Density supported on all of D: (x1(1-x1) x2(1-x2))^power times a seeded smooth factor.

    The polynomial is the one of Table globconv1 (power 3); it vanishes on the
    boundary of D only, so the zero extension needs a period b >= 1 + sqrt 2.
    Draw order: m ~ U{1..4}; then per term: frequencies f1, f2 ~ U[0.5, 3]
    (f1 then f2), phase p ~ U[0, 2 pi), amplitude A ~ N(0, 1).
    u = poly * (1 + 0.5 sum_i A_i cos(2 pi (f1 x1 + f2 x2) + p)).
    """
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 5))
    terms = []
    for _ in range(m):
        f1 = rng.uniform(0.5, 3.0)
        f2 = rng.uniform(0.5, 3.0)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        a = rng.normal()
        terms.append((f1, f2, ph, a))
    x1, x2 = grid(n)
    fac = np.ones((n, n))
    for f1, f2, ph, a in terms:
        fac += 0.5 * a * np.cos(2.0 * math.pi * (f1 * x1 + f2 * x2) + ph)
    return (x1 * (1.0 - x1) * x2 * (1.0 - x2)) ** power * fac


def disc_radius(seed: int) -> float:
    """Radius R ~ U[0.15, 0.35] of a piecewise-constant disc density (centre (0.5, 0.5))."""
    rng = np.random.default_rng(seed)
    return float(rng.uniform(0.15, 0.35))


def contrast(n: int, amplitude: float = 0.5) -> np.ndarray:
    """Smooth contrast m = amplitude * cut on the disc r < 0.4 about (0.5, 0.5)."""
    return amplitude * cutoff(n)


def plane_wave_angle(seed: int) -> float:
    rng = np.random.default_rng(seed)
    return float(rng.uniform(0.0, 2.0 * math.pi))


def plane_wave(n: int, kappa: float, theta: float) -> np.ndarray:
    """Incident field exp(i kappa d.x), d = (cos theta, sin theta), on the grid."""
    x1, x2 = grid(n)
    return np.exp(1j * kappa * (math.cos(theta) * x1 + math.sin(theta) * x2))


def random_field(shape, seed: int, complex_: bool = False) -> np.ndarray:
    """Unstructured N(0,1) samples (used for algebraic property tests)."""
    rng = np.random.default_rng(seed)
    if complex_:
        return rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return rng.normal(size=shape)


# Seeds of the benchmark workloads.
SEED_SMOOTH_BATCH = 1000      # smooth density i uses 1000 + i
SEED_DISC_BATCH = 1100        # disc density i uses 1100 + i
SEED_PRECISION = 2000         # 2048^2 precision study: 2000 + i
SEED_LS_ANGLE = 3000          # plane-wave angle: 3000 + kappa
SEED_TRACE = 4000             # serving arrival trace
SEED_FULL_SUPPORT = 5000      # period-3 densities on all of D: 5000 + i
