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


def _rect_antiderivative(x, y):
    """F with d2F/dx dy = log sqrt(x^2 + y^2):
    F = x y (log(x^2 + y^2) - 3)/2 + (x^2/2) atan(y/x) + (y^2/2) atan(x/y),
    each term continued by its limit 0 where it is 0 * (bounded)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = x * x + y * y
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(r2 > 0, x * y * (np.log(np.where(r2 > 0, r2, 1.0)) - 3.0) / 2.0, 0.0)
        t2 = np.where(x != 0, x * x / 2.0 * np.arctan(y / np.where(x != 0, x, 1.0)), 0.0)
        t3 = np.where(y != 0, y * y / 2.0 * np.arctan(x / np.where(y != 0, y, 1.0)), 0.0)
    return t1 + t2 + t3


def square_log_integral(lo: float, hi: float, x1, x2):
    """int_{[lo,hi]^2} log|x - y| dy, by the corner sum of the antiderivative above
    (the exact potential of the Poisson example with a discontinuous right-hand side)."""
    F = _rect_antiderivative
    return F(x1 - lo, x2 - lo) - F(x1 - lo, x2 - hi) - F(x1 - hi, x2 - lo) + F(x1 - hi, x2 - hi)


def helmholtz_radial_potential(profile, support: float, kappa: float, radii: np.ndarray) -> np.ndarray:
    """(A f)(r) = int g(x - y) f(|y - c|) dy for g = (i/4) H0^(1)(kappa |x|) and a radial f
    supported in s < support, at distance r = |x - c|.

    Graf's addition theorem expands H0^(1)(kappa |x - y|) in the angular harmonics
    H_m^(1)(kappa r_>) J_m(kappa r_<) e^{i m (theta - phi)}; integrating over the angle of y
    keeps only m = 0, so
        (A f)(r) = (i pi / 2) [H0(kappa r) int_0^r J0(kappa s) f(s) s ds
                               + J0(kappa r) int_r^support H0(kappa s) f(s) s ds],
    two 1D integrals computed here by adaptive quadrature (complex profiles allowed)."""
    from scipy import special

    radii = np.asarray(radii, dtype=np.float64)
    uniq, inv = np.unique(np.round(radii, 14), return_inverse=True)
    out = np.empty(uniq.shape, dtype=np.complex128)
    opts = dict(epsabs=1e-15, epsrel=1e-13, limit=400)

    def cquad(fun, lo, hi):
        if hi <= lo:
            return 0j
        re = integrate.quad(lambda s: complex(fun(s)).real, lo, hi, **opts)[0]
        im = integrate.quad(lambda s: complex(fun(s)).imag, lo, hi, **opts)[0]
        return re + 1j * im

    for i, r in enumerate(uniq):
        rr = min(r, support)
        inner = cquad(lambda s: special.j0(kappa * s) * profile(s) * s, 0.0, rr)
        outer = cquad(lambda s: special.hankel1(0, kappa * s) * profile(s) * s, rr, support)
        first = special.hankel1(0, kappa * r) * inner if r > 0 else 0.0
        out[i] = 0.5j * math.pi * (first + special.j0(kappa * r) * outer)
    return out[inv].reshape(radii.shape)
