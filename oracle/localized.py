"""Localised moments (Section 2.3) and the Yukawa kernel.

Test infrastructure only (see the package header).

With a smooth window eta_beta (1 on [0, beta/2], 0 beyond beta), the operator
splits as in eq. io_split into a convolution with the smooth kernel
g (1 - eta_beta) and one with the localised singular kernel g eta_beta:

* smooth part: the trapezoidal rule on the grid,
      T_i = h^2 sum_j g_s(|x_i - x_j|) u_j,   g_s = g (1 - eta_beta),  h = 1/n.
  With i - j in (-n, n)^2 this is a cyclic convolution of length nb, so in the
  form of eq. An its coefficients are the DFT of the kernel samples,
      Khat(k) = sum_{m in (-n, n)^2} h^2 g_s(|m| h) e^{-2 pi i k.m / nb}
  (real and even: a product of cosine transforms over m >= 0, with weight 2
  for m > 0).  g_s(0) = 0 since eta_beta(0) = 1.
* singular part: eq. An with the localised moments
      ghat_eta(k) = 2 pi int_0^beta g(rho) eta_beta(rho) J0(xi rho) rho d rho,
  xi = 2 pi |k| / b, computed after the substitution rho = beta tau^p by the
  trapezoidal rule in tau on [0, 1] with m intervals (the integrand vanishes
  to high order at both ends, so the trapezoidal rule is accurate).

The table of the localised scheme is ghat_eta(|k|) + Khat(k) on F_n, used in
place of ghat by scheme.apply.

Window: eta_beta(rho) = step((rho - beta/2) / (beta/2)) with the paper's own
smooth step kappa(t) = exp(2 e^(-1/t) / (t - 1)) (smoothing.step), the same
function as the window psi of Section 2.4.

Yukawa kernel g(x) = scale K0(kappa |x|) (Table yukawa uses scale = 1/(2 pi)).
Its moments truncated to B_a also have a closed form, from d/drho of
rho (xi J1(xi rho) K0(kappa rho) - kappa J0(xi rho) K1(kappa rho)) =
(xi^2 + kappa^2) rho J0(xi rho) K0(kappa rho) and rho kappa K1(kappa rho) -> 1:
    int_0^a rho K0(kappa rho) J0(xi rho) d rho
        = (1 + a xi J1(xi a) K0(kappa a) - a kappa J0(xi a) K1(kappa a)) / (xi^2 + kappa^2),
so ghat(k) = 2 pi scale times that; ``yukawa_global`` tabulates it for the
global scheme (a pin of the localised one).

Pins (tests/test_oracle_localized.py): ghat_eta against 30-digit mpmath
quadrature; the Yukawa closed form against mpmath quadrature; the localised
scheme against the global closed-form schemes (log and Yukawa); Table yukawa.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from .moments import frequencies
from .smoothing import step


def eta(rho, beta: float) -> np.ndarray:
    """eta_beta: 1 for rho <= beta/2, 0 for rho >= beta, C-infinity between."""
    rho = np.asarray(rho, dtype=np.float64)
    return step((rho - 0.5 * beta) / (0.5 * beta))


def yukawa(rho, kappa: float, scale: float = 1.0) -> np.ndarray:
    """g(rho) = scale K0(kappa rho)."""
    return scale * special.k0(kappa * np.asarray(rho, dtype=np.float64))


def ghat_eta(g, kabs: np.ndarray, beta: float, b: float, p: int = 4, m: int = 128) -> np.ndarray:
    """Localised moments 2 pi int_0^beta g eta_beta J0(xi rho) rho d rho, rho = beta tau^p, trapezoid in tau."""
    tau = np.arange(m + 1, dtype=np.float64) / m
    w = np.full(m + 1, 1.0 / m)
    w[0] = w[-1] = 0.5 / m
    rho = beta * tau ** p
    jac = p * beta * tau ** (p - 1)                  # d rho / d tau
    f = np.zeros(m + 1)
    f[1:] = g(rho[1:]) * eta(rho[1:], beta) * rho[1:] * jac[1:]   # -> 0 at tau = 0 (rho log rho)
    kabs = np.asarray(kabs, dtype=np.float64)
    xi = 2.0 * math.pi * kabs.reshape(-1) / b
    out = 2.0 * math.pi * (special.j0(np.outer(xi, rho)) @ (w * f))
    return out.reshape(kabs.shape)


def khat_smooth(g, n: int, b: int, beta: float) -> np.ndarray:
    """DFT on F_n (nb x nb, FFT-bin order) of the trapezoid samples h^2 g (1 - eta_beta) on (-n, n)^2."""
    nb = n * b
    h = 1.0 / n
    mm = np.arange(n, dtype=np.float64)
    m1, m2 = np.meshgrid(mm, mm, indexing="ij")
    r = h * np.hypot(m1, m2)
    ks = np.zeros((n, n))
    nz = r > 0
    ks[nz] = h * h * g(r[nz]) * (1.0 - eta(r[nz], beta))
    wgt = np.where(mm == 0, 1.0, 2.0)
    ks *= np.outer(wgt, wgt)
    k = frequencies(nb).astype(np.float64)
    c = np.cos(2.0 * math.pi * np.outer(k, mm) / nb)  # (nb, n)
    return c @ ks @ c.T


def nodes(n: int, beta: float) -> int:
    """Trapezoid intervals in tau for ghat_eta: enough to follow J0(xi rho) up to the largest
    xi = pi sqrt(2) n on F_n (about a quarter radian per step where rho = beta tau^4 is
    stretched most), and at least 768, which resolves the window's step to about 1e-15
    (the smooth step is flat but not analytic at its ends, so the rule converges faster
    than any power but slower than geometrically)."""
    return max(768, int(math.ceil(4.0 * beta * math.pi * math.sqrt(2.0) * n)))


def ghat_table_local(g, n: int, b: int, beta: float, p: int = 4, m: int | None = None) -> np.ndarray:
    """Table of the localised scheme: ghat_eta(|k|) + Khat(k) for k in F_n (nb x nb, FFT-bin order)."""
    m = nodes(n, beta) if m is None else m
    nb = n * b
    k = frequencies(nb).astype(np.int64)
    kabs = np.sqrt((k[:, None] ** 2 + k[None, :] ** 2).astype(np.float64))
    return ghat_eta(g, kabs, beta, b, p, m) + khat_smooth(g, n, b, beta)


def yukawa_global(kabs: np.ndarray, a: float, b: float, kappa: float, scale: float = 1.0) -> np.ndarray:
    """Closed-form moments of scale K0(kappa |x|) truncated to B_a (see the module header)."""
    kabs = np.asarray(kabs, dtype=np.float64)
    xi = 2.0 * math.pi * kabs / b
    num = 1.0 + a * xi * special.j1(xi * a) * special.k0(kappa * a) - a * kappa * special.j0(xi * a) * special.k1(kappa * a)
    return 2.0 * math.pi * scale * num / (xi * xi + kappa * kappa)


def yukawa_global_table(n: int, b: int, a: float, kappa: float, scale: float = 1.0) -> np.ndarray:
    nb = n * b
    k = frequencies(nb).astype(np.int64)
    kabs = np.sqrt((k[:, None] ** 2 + k[None, :] ** 2).astype(np.float64))
    return yukawa_global(kabs, a, b, kappa, scale)
