"""Pins of the oracle's discrete operator A_n (oracle/scheme.py)."""
import math

import numpy as np
import pytest

import synth
from oracle import metrics, moments, scheme
from tests import closed_forms as cf

B = 2
A2 = (B + math.sqrt(2) / 2 - 0.5) / 2      # b = 2, density in a disc about the centre
LAPLACE = moments.Kernel("log", -1.0 / (2.0 * math.pi))


def _apply(u, kernel, b, a):
    n = u.shape[-1]
    return scheme.apply(u, moments.ghat_table(kernel, n, b, a), b)


@pytest.mark.parametrize("n,b", [(6, 2), (5, 3), (4, 4)])
def test_apply_equals_quadrature_weights_bruteforce(n, b):
    # eq. An evaluated by FFT must equal eqs. quad/quad_wts summed term by term.
    rng = np.random.default_rng(n)
    u = rng.normal(size=(n, n))
    a = (math.sqrt(2) + b - 1) / 2 if b >= 3 else A2
    g = moments.ghat_table(moments.Kernel("power", 1.0, -0.5), n, b, a)
    full = scheme.apply(u, g, b)
    idx = [(0, 0), (n - 1, 2), (2, n - 1), (n // 2, n // 2)]
    pts = np.array([[i / n, j / n] for i, j in idx])
    brute = scheme.apply_weights(u, g, b, pts)
    for (i, j), v in zip(idx, brute):
        assert abs(full[i, j] - v) < 1e-13 * np.max(np.abs(full))


@pytest.mark.parametrize("n,b,kname", [(8, 2, "power"), (6, 3, "log"), (8, 2, "helmholtz")])
def test_apply_at_equals_quadrature_weights_off_grid(n, b, kname):
    # eq. An at off-grid points (series form) equals the quadrature-weight sum
    # of eqs. quad/quad_wts, term by term; targets also outside D and on it
    rng = np.random.default_rng(100 + n)
    u = rng.normal(size=(n, n)) + (1j * rng.normal(size=(n, n)) if kname == "helmholtz" else 0.0)
    a = (math.sqrt(2) + b - 1) / 2 if b >= 3 else A2
    kern = {"power": moments.Kernel("power", 1.0, -0.5), "log": moments.Kernel("log", 1.0),
            "helmholtz": moments.Kernel("helmholtz", 1.0, 0.0, 20.0)}[kname]
    g = moments.ghat_table(kern, n, b, a)
    pts = np.concatenate([rng.uniform(0.0, 1.0, size=(5, 2)), [[0.0, 0.0], [1.0, 0.5], [-0.3, 1.7]]])
    at = scheme.apply_at(u, g, b, pts)
    brute = scheme.apply_weights(u, g, b, pts)
    assert np.max(np.abs(at - brute)) < 1e-12 * np.max(np.abs(brute))
    # off the grid the sum over the asymmetric F_n is complex even for real u
    if kname != "helmholtz":
        assert np.max(np.abs(at[:5].imag)) > 1e-6 * np.max(np.abs(at))


def test_apply_at_grid_points_equals_apply():
    n, b = 16, 2
    u = synth.smooth_density(n, 3)
    g = moments.ghat_table(moments.Kernel("log", 1.0), n, b, A2)
    full = scheme.apply(u, g, b)
    idx = [(0, 0), (3, 11), (15, 15), (8, 0)]
    pts = np.array([[i / n, j / n] for i, j in idx])
    at = scheme.apply_at(u, g, b, pts)
    for (i, j), v in zip(idx, at):
        assert abs(full[i, j] - v) < 1e-13 * np.max(np.abs(full))
        assert abs(v.imag) < 1e-13 * np.max(np.abs(full))


def test_apply_matches_numpy_fft():
    n = 32
    u = synth.smooth_density(n, 5)
    g = moments.ghat_table(moments.Kernel("log", 1.0), n, B, A2)
    ue = np.zeros((n * B, n * B))
    ue[:n, :n] = u
    ref = np.fft.ifft2(g * np.fft.fft2(ue))[:n, :n]
    got = scheme.apply(u, g, B)
    assert metrics.rel_linf(got, ref) < 1e-14


def test_config0_bump_against_newton_formula():
    # Radial bump with g = -(1/2pi) log: super-algebraic convergence to the
    # Newton potential (Section 3.1 reports super-algebraic rates for C-infinity data).
    errs = []
    for n in (32, 64, 128):
        u = synth.bump_density(n)
        got = np.real(_apply(u, LAPLACE, B, A2))
        exact = cf.newton_log_potential(cf.bump_profile(), 0.4, synth.radius(n))
        errs.append(metrics.rel_linf(got, exact))
    assert errs[0] < 1e-4 and errs[1] < 1e-6 and errs[2] < 1e-8
    assert errs[0] / errs[1] > 50 and errs[1] / errs[2] > 50


def test_spectral_laplacian_recovers_density():
    # -Delta(A u) = u in D for the fundamental solution g = -(1/2pi) log.  The
    # spectral Laplacian of A_n u multiplies ghat(k) by (2 pi |k| / b)^2; the
    # truncation layer terms J0(xi a) + a log(a) xi J1(xi a) only see the
    # (slowly decaying) high frequencies of the bump, so the error shrinks with n.
    errs = []
    for n in (32, 64, 128):
        u = synth.bump_density(n)
        g = moments.ghat_table(LAPLACE, n, B, A2)
        k = moments.frequencies(n * B).astype(float)
        xi2 = (2 * math.pi / B) ** 2 * (k[:, None] ** 2 + k[None, :] ** 2)
        lap = np.real(scheme.apply(u, xi2 * g, B))
        errs.append(metrics.rel_linf(lap, u))
    assert errs[2] < 3e-6
    assert errs[0] / errs[1] > 5 and errs[1] / errs[2] > 5


def test_linearity_shift_transpose_realness():
    n = 32
    u1 = synth.smooth_density(n, 11)
    u2 = synth.smooth_density(n, 12)
    g = moments.ghat_table(moments.Kernel("power", 1.0, -0.5), n, B, A2)
    r1 = scheme.apply(u1, g, B)
    r2 = scheme.apply(u2, g, B)
    r12 = scheme.apply(2.0 * u1 - 3.0 * u2, g, B)
    scale = np.max(np.abs(r12))
    assert np.max(np.abs(r12 - (2 * r1 - 3 * r2))) < 1e-13 * scale
    # transpose equivariance (ghat(k1, k2) = ghat(k2, k1))
    assert np.max(np.abs(scheme.apply(u1.T, g, B) - r1.T)) < 1e-13 * scale
    # realness for a real kernel and density
    assert np.max(np.abs(r1.imag)) < 1e-15 * scale
    # circular shift equivariance: the operator is a circular convolution on the
    # nb-periodic grid; shifting a density that stays inside G_n shifts the result.
    nb = n * B
    ue = np.zeros((nb, nb))
    ue[:n, :n] = u1
    sh = np.roll(ue, (3, -2), axis=(0, 1))
    full = np.fft.ifft2(g * np.fft.fft2(ue))
    full_sh = np.fft.ifft2(g * np.fft.fft2(sh))
    assert np.max(np.abs(np.roll(full, (3, -2), axis=(0, 1)) - full_sh)) < 1e-13 * scale
    # and the oracle apply agrees with that circular convolution on G_n
    assert np.max(np.abs(full[:n, :n] - r1)) < 1e-13 * scale


def _gauss_e1(n):
    # Table globconv_gauss density, centred at (0.5, 0.5) (the printed |y| reads as |y - c|).
    s = 0.05
    x1, x2 = synth.grid(n)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2
    return np.exp(-r2 / (2 * s * s)) / (2 * math.pi * s * s)


def test_table_globconv_gauss_log_column_rates():
    # Table globconv_gauss, g = log|x|, b = 3: eps_n = 2.3e-1, 1.3e-3, 3.8e-9 for
    # n = 8, 16, 32 (super-algebraic).  The exact reference is Newton's formula
    # (the Gaussian is below 1e-21 outside r = 0.5).
    b = 3
    a = (math.sqrt(2) + b - 1) / 2
    kern = moments.Kernel("log", 1.0)
    s = 0.05
    prof = lambda r: math.exp(-r * r / (2 * s * s)) / (2 * math.pi * s * s)
    errs = {}
    for n in (8, 16, 32):
        got = np.real(_apply(_gauss_e1(n), kern, b, a))
        exact = -2 * math.pi * cf.newton_log_potential(prof, 0.5, synth.radius(n))
        errs[n] = metrics.rel_linf(got, exact)
    assert 0.02 < errs[8] < 2.0
    assert 1e-4 < errs[16] < 1e-2
    assert 3e-10 < errs[32] < 4e-8          # printed 3.8e-9
    assert metrics.noc(errs[16], errs[32]) > 12


def test_table_globconv1_rate_power_kernel():
    # Table globconv1: u = (x1(1-x1)x2(1-x2))^3, g = |x|^-1/2, b = 3: noc ~ 4.0.
    b = 3
    a = (math.sqrt(2) + b - 1) / 2
    kern = moments.Kernel("power", 1.0, -0.5)

    def dens(n):
        x1, x2 = synth.grid(n)
        return (x1 * (1 - x1) * x2 * (1 - x2)) ** 3

    nref = 64
    ref = np.real(_apply(dens(nref), kern, b, a))
    errs = []
    for n in (8, 16):
        got = np.real(_apply(dens(n), kern, b, a))
        step = nref // n
        errs.append(metrics.rel_linf(got, ref[::step, ::step]))
    rate = metrics.noc(errs[0], errs[1])
    assert 3.4 < rate < 4.8            # printed: 4.8 then 4.1 between n = 4..16
