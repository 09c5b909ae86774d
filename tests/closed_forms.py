"""Exact potentials used as pins (computed independently of the oracle's scheme).

Newton's formula: for g = -(1/2pi) log|x| and a density that depends only on
s = |y - c|, the potential at distance r from c is
    (Au)(r) = - int_0^inf s u(s) log(max(r, s)) ds,
because the circle average of log|x - y| over |y - c| = s equals log max(r, s).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def newton_log_potential(profile, support: float, radii: np.ndarray) -> np.ndarray:
    """-(1/2pi) log kernel potential of a radial density ``profile(s)`` (s < support)."""
    radii = np.asarray(radii, dtype=np.float64)
    uniq, inv = np.unique(np.round(radii, 15), return_inverse=True)
    out = np.empty(uniq.shape)
    opts = dict(epsabs=1e-17, epsrel=1e-14, limit=400)
    total_mass, _ = integrate.quad(lambda s: s * profile(s), 0.0, support, **opts)
    for i, r in enumerate(uniq):
        if r >= support:
            out[i] = -math.log(r) * total_mass
            continue
        inner = 0.0
        if r > 0:
            inner, _ = integrate.quad(lambda s: s * profile(s), 0.0, r, **opts)
        outer, _ = integrate.quad(lambda s: s * profile(s) * math.log(s), r, support, **opts)
        out[i] = -(math.log(r) * inner if r > 0 else 0.0) - outer
    return out[inv].reshape(radii.shape)


def bump_profile(rho: float = 0.4):
    def f(s):
        if s >= rho:
            return 0.0
        t = 1.0 - (s / rho) ** 2
        return math.exp(1.0 - 1.0 / t)
    return f


def disc_log_potential(radius: float, r: np.ndarray) -> np.ndarray:
    """-(1/2pi) log potential of the indicator of a disc of the given radius."""
    r = np.asarray(r, dtype=np.float64)
    inside = radius ** 2 / 4 - r ** 2 / 4 - radius ** 2 / 2 * math.log(radius)
    with np.errstate(divide="ignore"):
        outside = -radius ** 2 / 2 * np.log(np.where(r > 0, r, 1.0))
    return np.where(r <= radius, inside, outside)
