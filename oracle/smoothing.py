"""Fourier smoothing of densities with jumps (Section 2.4).

Test infrastructure only (see the package header).

For u = u_tilde * chi_Omega with a smooth u_tilde, the paper replaces the
indicator chi_Omega by its truncated Fourier series chi^n on F_n and a smooth
window psi (1 on Omega, 0 on the boundary of D), eqs. ls1 and tfs, and applies
A_n to u_tilde * chi^n * psi.

Readings taken here (the paper is silent or garbled on these points):

* Period of the series: the paper prints exp(2 pi i k.x) with k running over
  F_n (nb^2 frequencies); it is read as period b,
      chi^n(x) = sum_{k in F_n} chihat(k) exp(2 pi i k.x / b),
      chihat(k) = b^-2 int_Omega exp(-2 pi i k.y / b) dy,
  which makes the series the b-periodic Fourier series of the extended indicator.
* The window psi is only pictured.  It is built from the paper's own smooth
  step kappa_step(t) = exp(2 e^(-1/t) / (t - 1)) on (0, 1) (given with the smooth
  refractive index of the scattering examples): psi(r) = 1 for r <= R1,
  kappa_step((r - R1)/(R2 - R1)) for R1 < r < R2, 0 for r >= R2, with r the
  distance to the shape's centre.
* The smoothed density is taken as the real part of u_tilde * chi^n * psi.  For
  the disc centred at (0.5, 0.5) with n divisible by 4 the series is exactly real
  (the k = -nb/2 terms equal their k = +nb/2 mirror images).

Pins (tests/test_oracle_smoothing_ls.py): chihat (disc and square) against
2D quadrature of the indicator; chi^n against a brute-force sum of the series
at sample points; the windows' values (1 on Omega, 0 beyond the ramp or on
the boundary of D, the smooth step's value at mid-ramp from 30-digit
arithmetic, monotone, radial or separable); the disc potential closed form
for g = -(1/2pi) log with second-order convergence; the square [0.3, 0.7]^2
against its exact log potential (corner sum of an antiderivative of log|x|):
Table conv_FS at b = 3 with the tensor window (second order, magnitudes
within a small factor of the printed ones, the plain indicator first order)
and the radial-window square at b = 2 (second order).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import fft as _fft
from .moments import frequencies


def step(t: np.ndarray) -> np.ndarray:
    """kappa_step(t) = exp(2 e^(-1/t)/(t - 1)): 1 for t <= 0, 0 for t >= 1, C-infinity."""
    t = np.asarray(t, dtype=np.float64)
    out = np.where(t <= 0.0, 1.0, 0.0)
    mid = (t > 0.0) & (t < 1.0)
    tm = t[mid]
    with np.errstate(over="ignore", under="ignore"):
        out[mid] = np.exp(2.0 * np.exp(-1.0 / tm) / (tm - 1.0))
    return out


def radial_window(n: int, centre, r1: float, r2: float) -> np.ndarray:
    t = np.arange(n) / n
    x1, x2 = np.meshgrid(t, t, indexing="ij")
    r = np.hypot(x1 - centre[0], x2 - centre[1])
    return step((r - r1) / (r2 - r1))


def chihat_disc(n: int, b: int, centre, radius: float) -> np.ndarray:
    """b^-2 int_disc exp(-2 pi i k.y/b) dy on F_n in FFT-bin order (nb x nb)."""
    nb = n * b
    k = frequencies(nb).astype(np.int64)
    k1, k2 = np.meshgrid(k, k, indexing="ij")
    kabs = np.sqrt((k1 ** 2 + k2 ** 2).astype(np.float64))
    out = np.empty(kabs.shape, dtype=np.float64)
    zero = kabs == 0
    out[zero] = math.pi * radius * radius / (b * b)
    kk = kabs[~zero]
    out[~zero] = radius / (b * kk) * special.j1(2.0 * math.pi * kk * radius / b)
    phase = np.exp(-2j * math.pi * (k1 * centre[0] + k2 * centre[1]) / b)
    return out * phase


def chihat_square(n: int, b: int, lo: float, hi: float) -> np.ndarray:
    """b^-2 int_[lo,hi]^2 exp(-2 pi i k.y/b) dy on F_n in FFT-bin order (separable)."""
    nb = n * b
    k = frequencies(nb).astype(np.float64)
    one = np.empty(nb, dtype=np.complex128)
    z = k == 0
    one[z] = hi - lo
    w = 2.0 * math.pi * k[~z] / b
    one[~z] = (np.exp(-1j * w * lo) - np.exp(-1j * w * hi)) / (1j * w)
    return np.outer(one, one) / (b * b)


def series_on_grid(coef: np.ndarray, n: int, b: int) -> np.ndarray:
    """chi^n(x_j) = sum_{k in F_n} coef(k) exp(2 pi i k.j/(nb)) for j in G_n (complex)."""
    full = _fft.fft2(coef, inverse=True)
    return full[:n, :n]


def smoothed_disc_density(n: int, b: int, radius: float, centre=(0.5, 0.5),
                          r2: float = 0.39, u_tilde: np.ndarray | None = None) -> np.ndarray:
    """Re(u_tilde * chi^n * psi) for a disc indicator; psi ramps from r=radius to r=r2."""
    chi = series_on_grid(chihat_disc(n, b, centre, radius), n, b)
    psi = radial_window(n, centre, radius, r2)
    ut = 1.0 if u_tilde is None else u_tilde
    return np.real(ut * chi * psi)


def smoothed_square_density(n: int, b: int, lo: float, hi: float, r1: float, r2: float,
                            centre=(0.5, 0.5), u_tilde: np.ndarray | None = None) -> np.ndarray:
    """Re(u_tilde * chi^n * psi) for the square [lo, hi]^2 with a radial window psi."""
    chi = series_on_grid(chihat_square(n, b, lo, hi), n, b)
    psi = radial_window(n, centre, r1, r2)
    ut = 1.0 if u_tilde is None else u_tilde
    return np.real(ut * chi * psi)


def tensor_window(n: int, lo: float, hi: float) -> np.ndarray:
    """Product of 1D smooth steps: 1 on [lo, hi]^2, 0 on the boundary of D.

    The window of Table conv_FS's square, whose support is all of D (so b = 3)."""
    t = np.arange(n) / n
    left = step((lo - t) / lo)            # 1 at t >= lo, 0 at t = 0
    right = step((t - hi) / (1.0 - hi))   # 1 at t <= hi, 0 at t = 1
    w = left * right
    return np.outer(w, w)
