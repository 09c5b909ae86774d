"""The discrete convolution operator A_n (Section 2.1).

Test infrastructure only (see the package header).

Given grid samples u_j = u(j/n), j in G_n = [0, n)^2, a period b and the
moments ghat(k) on F_n (an nb x nb set of frequencies, nb = n b), eq. An reads

    (A_n u)(x) = sum_{k in F_n} ghat(k) uhat_{e,n}(k) exp(2 pi i k.x / b),
    uhat_{e,n}(k) = (nb)^-2 sum_{j in G_n} u_j exp(-2 pi i k.j / nb)        (trapezoid)

and is evaluated at the grid points x_i = i/n, i in G_n.  ``apply`` follows
those steps in order: zero-extend the samples to the nb x nb periodic grid
(eq. fc_discrete), take the forward DFT with the (nb)^-2 factor, multiply by
ghat, take the inverse DFT at the grid points of D and restrict to G_n.

``apply_at`` reads eq. An at arbitrary (also off-grid) targets, and
``apply_weights`` is the quadrature form of eqs. quad / quad_wts:
(A_n u)(x) = sum_j w_j^n(x) u_j with
w_j^n(x) = (nb)^-2 sum_k ghat(k) exp(2 pi i k.(x - x_j)/b),
evaluated by brute force for any (also off-grid) target x.

Pins (tests/test_oracle_scheme.py): apply == apply_weights (O(N^2) brute
force) on small grids; apply_at == apply_weights at off-grid targets and ==
apply at grid points; agreement with a numpy.fft evaluation (third-party);
the Laplace potential of a radial bump from Newton's formula (a 1D integral);
Delta(A_n u) = -u for g = -(1/2pi) log via the spectral identity of the
truncated kernel; linearity, circular shift and transpose equivariance; the
convergence rates printed in Tables globconv_gauss / globconv1 / conv_FS.
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft
from .moments import frequencies


def extend(u: np.ndarray, b: int) -> np.ndarray:
    """Zero extension of the n x n samples to the nb x nb grid of D_e = [0, b]^2."""
    n = u.shape[-1]
    nb = n * b
    ue = np.zeros(u.shape[:-2] + (nb, nb), dtype=np.complex128)
    ue[..., :n, :n] = u
    return ue


def apply(u: np.ndarray, ghat_full: np.ndarray, b: int) -> np.ndarray:
    """(A_n u)(x_i), i in G_n, for samples u (shape (..., n, n)); complex result.

    ``ghat_full`` holds ghat(k) for k in F_n in FFT-bin order (nb x nb).
    """
    n = u.shape[-1]
    nb = n * b
    ue = extend(u, b)
    uhat = _fft.fft2(ue) / float(nb * nb)           # trapezoidal coefficients
    prod = ghat_full * uhat                          # multiply by the moments
    full = _fft.fft2(prod, inverse=True)             # sum_k ... exp(+2 pi i k.j / nb)
    return full[..., :n, :n]                         # restrict to G_n


def apply_at(u: np.ndarray, ghat_full: np.ndarray, b: int, targets: np.ndarray) -> np.ndarray:
    """(A_n u)(x) for arbitrary targets x (shape (m, 2)): eq. An read at x.

    The coefficients ghat(k) uhat_{e,n}(k) on F_n are formed as in ``apply``;
    the series sum_k c(k) exp(2 pi i k.x / b) is then summed at each target,
    over k2 first (a matrix product with the k2 exponentials) and then over k1.
    F_n = [-nb/2, nb/2)^2 is not symmetric, so the result is complex even for
    real u off the grid.
    """
    n = u.shape[-1]
    nb = n * b
    coef = ghat_full * (_fft.fft2(extend(u, b)) / float(nb * nb))
    k = frequencies(nb).astype(np.float64)
    out = np.empty(len(targets), dtype=np.complex128)
    for t, (x1, x2) in enumerate(targets):
        e1 = np.exp(2j * np.pi * k * x1 / b)
        e2 = np.exp(2j * np.pi * k * x2 / b)
        out[t] = e1 @ (coef @ e2)
    return out


def apply_weights(u: np.ndarray, ghat_full: np.ndarray, b: int,
                  targets: np.ndarray) -> np.ndarray:
    """Quadrature form: sum_j w_j^n(x) u_j for targets x (shape (m, 2)); brute force."""
    n = u.shape[-1]
    nb = n * b
    k = frequencies(nb).astype(np.float64)
    k1, k2 = np.meshgrid(k, k, indexing="ij")
    k1 = k1.ravel()
    k2 = k2.ravel()
    g = ghat_full.ravel()
    jj = np.arange(n) / n
    xj1, xj2 = np.meshgrid(jj, jj, indexing="ij")
    xj1 = xj1.ravel()
    xj2 = xj2.ravel()
    uf = u.reshape(-1)
    out = np.empty(len(targets), dtype=np.complex128)
    for t, (x1, x2) in enumerate(targets):
        d1 = x1 - xj1
        d2 = x2 - xj2
        phase = np.exp(2j * np.pi * (np.outer(d1, k1) + np.outer(d2, k2)) / b)
        w = phase @ g / float(nb * nb)
        out[t] = np.dot(w, uf)
    return out
