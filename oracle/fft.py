"""Discrete Fourier transforms for the oracle (own code, no FFT library).

Test infrastructure only (see the package header).

Convention (the one used by the trapezoidal coefficients of Section 2.1):
forward  X[k] = sum_j x[j] exp(-2 pi i j k / N)   (unnormalised)
inverse  x[j] = sum_k X[k] exp(+2 pi i j k / N)   (unnormalised)

``dft`` is the O(N^2) definition.  ``fft`` is a recursive mixed-radix
decimation-in-time transform: for N = r * M it transforms the r decimated
subsequences x[q::r] (length M), multiplies by exp(-2 pi i q k / N) and
combines them with an r-point DFT.  Radices 4, 2, 3, 5 are peeled in that
order; any other prime factor is handled by the O(N^2) definition.

Pins (tests/test_oracle_fft.py): fft == dft to rounding for many lengths,
agreement with numpy.fft as an independent third-party implementation, and
Parseval / shift theorem identities.
"""
from __future__ import annotations

import numpy as np


def dft(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Naive DFT along the last axis (the definition written out)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    j = np.arange(n)
    sign = 1.0 if inverse else -1.0
    # Reduce j*k modulo n before forming the angle to keep the phase exact.
    mat = np.exp(sign * 2j * np.pi * ((j[:, None] * j[None, :]) % n) / n)
    return x @ mat.T


def _radix(n: int) -> int:
    for r in (4, 2, 3, 5):
        if n % r == 0:
            return r
    return n


def _fft_last(x: np.ndarray, sign: float) -> np.ndarray:
    n = x.shape[-1]
    if n == 1:
        return x.copy()
    r = _radix(n)
    if r == n:
        # Prime length (or r itself): definition.
        j = np.arange(n)
        mat = np.exp(sign * 2j * np.pi * ((j[:, None] * j[None, :]) % n) / n)
        return x @ mat.T
    m = n // r
    lead = x.shape[:-1]
    # Subsequence q holds x[q], x[q + r], ..., i.e. element j = j' r + q.
    sub = x.reshape(lead + (m, r))
    sub = np.moveaxis(sub, -1, -2)                      # (..., r, m)
    y = _fft_last(np.ascontiguousarray(sub), sign)      # DFT_m of each subsequence
    q = np.arange(r)[:, None]
    kp = np.arange(m)[None, :]
    tw = np.exp(sign * 2j * np.pi * ((q * kp) % n) / n)  # exp(-+2 pi i q k'/N)
    z = y * tw
    # X[k' + m s] = sum_q exp(-+2 pi i q s / r) z[q, k']
    s = np.arange(r)
    small = np.exp(sign * 2j * np.pi * ((s[:, None] * s[None, :]) % r) / r)  # [s, q]
    out = np.tensordot(z, small, axes=([-2], [1]))      # (..., m, s)
    out = np.moveaxis(out, -1, -2)                      # (..., s, m): index k = s m + k'
    return out.reshape(lead + (n,))


def fft(x: np.ndarray, axis: int = -1, inverse: bool = False) -> np.ndarray:
    """Unnormalised forward (or inverse) DFT along ``axis`` by the mixed-radix recursion."""
    x = np.asarray(x, dtype=np.complex128)
    xm = np.moveaxis(x, axis, -1)
    out = _fft_last(np.ascontiguousarray(xm), 1.0 if inverse else -1.0)
    return np.moveaxis(out, -1, axis)


def fft2(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Unnormalised 2D transform over the last two axes."""
    return fft(fft(x, axis=-1, inverse=inverse), axis=-2, inverse=inverse)
