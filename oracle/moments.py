"""Kernel moments ghat(k) for radially symmetric kernels (Section 2.2).

Test infrastructure only (see the package header).

For a radial kernel g truncated to the ball B_a(0), eq. ghat gives
    ghat(k) = 2 pi int_0^a g(rho) J0(xi rho) rho d rho,   xi = 2 pi |k| / b.

Kernels (``scale`` multiplies g; the paper's closed forms are quoted for the
normalisations named below and rescaled here):

* ``log``:        g(x) = scale * log|x|.  Closed form of Section 2.2 for
                  -(1/2pi) log|x|, multiplied by -2 pi * scale.
* ``helmholtz``:  g(x) = scale * (i/4) H0^(1)(kappa |x|).  Closed form of
                  Section 2.2 with two readings: the |k| = 0 line uses
                  -2/(kappa pi) (the printed +2/(kappa pi) is not the k -> 0
                  limit of the generic line and disagrees with quadrature), and
                  the exact-resonance line is used when |xi - kappa| <= 1e-9 kappa.
* ``power``:      g(x) = scale * |x|^gamma, -2 < gamma < 0.  The paper gives a
                  Lommel-function closed form; the oracle instead evaluates the
                  defining radial integral directly: the termwise-integrated
                  power series of J0 on the first half period (which carries the
                  rho^(1+gamma) singularity exactly), and composite
                  Gauss-Legendre panels no longer than half a period of
                  J0(xi rho) on the rest.  This shares nothing with the GPU's
                  Fejer/substitution rule.

Pins (tests/test_oracle_moments.py): 30-digit mpmath quadrature of the
defining integral at sampled |k| for every family; the paper's Lommel closed
form (via mpmath.lommels2) for power kernels; the Struve closed form for
gamma = -1; the Helmholtz resonance line and the k -> 0 limit.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import special


@dataclass(frozen=True)
class Kernel:
    family: str            # "log" | "power" | "helmholtz"
    scale: float = 1.0
    gamma: float = 0.0     # power kernels
    kappa: float = 0.0     # Helmholtz


def log_paper(kabs: np.ndarray, a: float, b: float) -> np.ndarray:
    """ghat for g = -(1/2pi) log|x| (Section 2.2, Laplace kernel)."""
    kabs = np.asarray(kabs, dtype=np.float64)
    xi = 2.0 * math.pi * kabs / b
    out = np.empty_like(xi)
    zero = kabs == 0
    out[zero] = a * a / 4.0 * (1.0 - 2.0 * math.log(a))
    x = xi[~zero]
    z = x * a
    out[~zero] = -a * math.log(a) * special.j1(z) / x + (1.0 - special.j0(z)) / (x * x)
    return out


def helmholtz_paper(kabs: np.ndarray, a: float, b: float, kappa: float,
                    resonance_tol: float = 1e-9) -> np.ndarray:
    """ghat for g = (i/4) H0^(1)(kappa |x|) (Section 2.2, Helmholtz kernel)."""
    kabs = np.asarray(kabs, dtype=np.float64)
    xi = 2.0 * math.pi * kabs / b
    ka = kappa * a
    h0 = special.hankel1(0, ka)
    h1 = special.hankel1(1, ka)
    out = np.empty(xi.shape, dtype=np.complex128)
    zero = kabs == 0
    # |k| = 0 (sign of the last term read as -2/(kappa pi)).
    out[zero] = math.pi / (2.0 * kappa) * (1j * a * special.j1(ka) - a * special.y1(ka)
                                            - 2.0 / (kappa * math.pi))
    res = (~zero) & (np.abs(xi - kappa) <= resonance_tol * kappa)
    out[res] = 0.25j * math.pi * a * a * (special.j0(ka) * h0 + special.j1(ka) * h1)
    gen = (~zero) & (~res)
    x = xi[gen]
    z = x * a
    num = z * special.j1(z) * h0 - ka * special.j0(z) * h1 - 2j / math.pi
    out[gen] = 0.5j * math.pi * num / (x * x - kappa * kappa)
    return out


def _radial_power_integral(xi: float, a: float, gamma: float) -> float:
    """int_0^a rho^(1+gamma) J0(xi rho) d rho.

    On [0, h], h = min(a, pi/xi), the power series of J0 is integrated term by
    term: int_0^h rho^beta J0(xi rho) d rho
        = h^(beta+1) sum_m (-1)^m (xi h / 2)^(2m) / ((m!)^2 (beta + 1 + 2m)),
    with xi h <= pi so the terms stay below 3 in size (no cancellation).
    On [h, a] composite 24-point Gauss-Legendre panels no longer than half a
    period of J0 integrate the smooth remainder.
    """
    beta = 1.0 + gamma
    half_period = math.pi / xi if xi > 0 else a
    h = min(a, half_period)
    q = (0.5 * xi * h) ** 2
    term = 1.0
    series = 1.0 / (beta + 1.0)
    m = 0
    while True:
        m += 1
        term *= -q / (m * m)
        add = term / (beta + 1.0 + 2 * m)
        series += add
        if abs(add) < 1e-18 * abs(series) and m > 3:
            break
    total = h ** (beta + 1.0) * series
    if h < a:
        npan = int(math.ceil((a - h) / half_period))
        edges = np.linspace(h, a, npan + 1)
        xg, wg = np.polynomial.legendre.leggauss(24)
        lo = edges[:-1][:, None]
        hi = edges[1:][:, None]
        rho = 0.5 * (hi - lo) * xg[None, :] + 0.5 * (hi + lo)
        f = rho ** beta * special.j0(xi * rho)
        total += float(np.sum(0.5 * (hi - lo)[:, 0] * (f @ wg)))
    return float(total)


def power_radial(kabs: np.ndarray, a: float, b: float, gamma: float) -> np.ndarray:
    """int_0^a rho^(1+gamma) J0(2 pi |k| rho / b) d rho for each |k| (unique values once)."""
    kabs = np.asarray(kabs, dtype=np.float64)
    flat = kabs.ravel()
    uniq, inv = np.unique(flat, return_inverse=True)
    vals = np.empty(uniq.shape)
    for i, kk in enumerate(uniq):
        xi = 2.0 * math.pi * kk / b
        if kk == 0:
            vals[i] = a ** (2.0 + gamma) / (2.0 + gamma)
        else:
            vals[i] = _radial_power_integral(xi, a, gamma)
    return vals[inv].reshape(kabs.shape)


def ghat(kernel: Kernel, kabs: np.ndarray, a: float, b: float) -> np.ndarray:
    """Moments of ``scale * g`` at |k| (array), per the kernel family."""
    if kernel.family == "log":
        return -2.0 * math.pi * kernel.scale * log_paper(kabs, a, b)
    if kernel.family == "power":
        if not (-2.0 < kernel.gamma < 0.0):
            raise ValueError("power kernel needs -2 < gamma < 0")
        return 2.0 * math.pi * kernel.scale * power_radial(kabs, a, b, kernel.gamma)
    if kernel.family == "helmholtz":
        if not kernel.kappa > 0:
            raise ValueError("Helmholtz kernel needs kappa > 0")
        return kernel.scale * helmholtz_paper(kabs, a, b, kernel.kappa)
    raise ValueError(f"unknown kernel family {kernel.family!r}")


def frequencies(nb: int) -> np.ndarray:
    """Integer frequency k of each FFT bin q in [0, nb): the set F_n of Section 2.1.

    For even nb, F_n = [-nb/2, nb/2): bin q < nb/2 holds k = q, otherwise k = q - nb
    (so bin nb/2 holds k = -nb/2).  For odd nb the symmetric range is used.
    """
    q = np.arange(nb)
    if nb % 2 == 0:
        return np.where(q < nb // 2, q, q - nb)
    return np.where(q <= (nb - 1) // 2, q, q - nb)


def ghat_table(kernel: Kernel, n: int, b: int, a: float) -> np.ndarray:
    """ghat(k) for every k in F_n, laid out in FFT-bin order, shape (nb, nb)."""
    nb = n * b
    k = frequencies(nb).astype(np.int64)
    # |k| from the exact integer k1^2 + k2^2 so equal radii give identical values.
    kabs = np.sqrt((k[:, None] ** 2 + k[None, :] ** 2).astype(np.float64))
    return ghat(kernel, kabs, a, b)
