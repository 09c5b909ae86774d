"""Lippmann-Schwinger Nystrom system and its solvers (Section 3.3).

Test infrastructure only (see the package header).

eq. descretls: u(x_j) + kappa^2 (A_n(m u))(x_j) = u_inc(x_j), j in G_n, with the
contrast m = 1 - mu and the Helmholtz kernel g = (i/4) H0^(1)(kappa |x|).

* ``matvec``      -- v -> v + kappa^2 A_n(m v) using ``scheme.apply``.
* ``dense_solve`` -- builds the N x N matrix column by column (N = n^2, tiny n
                     only) and solves it by LU (numpy.linalg.solve).
* ``gmres``       -- restarted GMRES(restart) from x0 = 0 with classical
                     Gram-Schmidt applied twice and Givens rotations on the
                     Hessenberg matrix; stops when the true relative residual
                     ||u_inc - K x|| / ||u_inc|| is at most ``tol`` (checked at
                     each restart; the Givens estimate triggers the check).
                     The paper only says "matrix-free GMRES"; these settings
                     are a reading.

Pins (tests/test_oracle_smoothing_ls.py):
* ``matvec`` against a manufactured radial solution: for a radial contrast m
  and a radial field u about the centre, A(m u) for the Helmholtz kernel is
  two 1D Bessel integrals (Graf's addition theorem keeps only the m = 0
  harmonic), computed by adaptive quadrature without the scheme; with
  u_inc := u + kappa^2 A(m u), ``matvec(u)`` -> u_inc and the solutions of
  ``dense_solve`` / ``gmres`` -> u at the scheme's super-algebraic rate,
  while the operator with the scattered term's sign flipped stays O(1) away;
* gmres agrees with dense_solve at n = 8, 16; the residual of the returned
  solution, recomputed with ``matvec``, meets tol; for m = 0 the solution is
  u_inc.
"""
from __future__ import annotations

import numpy as np

from . import scheme


def matvec(v: np.ndarray, m: np.ndarray, ghat_full: np.ndarray, b: int, kappa: float) -> np.ndarray:
    return v + kappa * kappa * scheme.apply(m * v, ghat_full, b)


def dense_solve(m, u_inc, ghat_full, b, kappa):
    n = m.shape[0]
    nn = n * n
    mat = np.empty((nn, nn), dtype=np.complex128)
    e = np.zeros(nn, dtype=np.complex128)
    for c in range(nn):
        e[:] = 0
        e[c] = 1
        mat[:, c] = matvec(e.reshape(n, n), m, ghat_full, b, kappa).ravel()
    return np.linalg.solve(mat, u_inc.ravel()).reshape(n, n)


def gmres(m, u_inc, ghat_full, b, kappa, tol=1e-12, restart=50, max_matvecs=5000):
    """Returns (x, info) with info = dict(matvecs, restarts, rel_residual, converged)."""
    shape = u_inc.shape
    f = u_inc.ravel().astype(np.complex128)
    fnorm = np.linalg.norm(f)
    x = np.zeros_like(f)

    def op(v):
        return matvec(v.reshape(shape), m, ghat_full, b, kappa).ravel()

    matvecs = 0
    restarts = 0
    if fnorm == 0:
        return x.reshape(shape), dict(matvecs=0, restarts=0, rel_residual=0.0, converged=True)
    r = f.copy()
    rel = 1.0
    while matvecs < max_matvecs:
        beta = np.linalg.norm(r)
        rel = beta / fnorm
        if rel <= tol:
            break
        V = np.zeros((restart + 1, f.size), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(restart):
            w = op(V[j])
            matvecs += 1
            for _ in range(2):                      # CGS, twice
                h = V[: j + 1].conj() @ w
                w = w - h @ V[: j + 1]
                H[: j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            # Apply previous rotations to the new column.
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            # New rotation zeroing H[j+1, j].
            a_, b_ = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a_) ** 2 + abs(b_) ** 2)
            if den == 0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j] = a_ / den
                sn[j] = b_ / den
                # rotation [[conj(c), conj(s)], [-s, c]] applied to (a, b) gives (den, 0)
                cs[j] = np.conj(cs[j])
                sn[j] = np.conj(sn[j])
            H[j, j] = cs[j] * a_ + sn[j] * b_
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k_used = j + 1
            if abs(g[j + 1]) / fnorm <= tol or matvecs >= max_matvecs:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + y @ V[:k_used]
        r = f - op(x)
        matvecs += 1
        restarts += 1
    rel = np.linalg.norm(r) / fnorm
    return x.reshape(shape), dict(matvecs=matvecs, restarts=restarts, rel_residual=float(rel),
                                  converged=bool(rel <= tol))
