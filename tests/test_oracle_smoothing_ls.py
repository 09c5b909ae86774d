"""Pins of the oracle's Fourier smoothing (oracle/smoothing.py) and LS solvers (oracle/ls.py)."""
import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle import ls, metrics, moments, scheme, smoothing
from tests import closed_forms as cf

B = 2
A2 = (B + math.sqrt(2) / 2 - 0.5) / 2
LAPLACE = moments.Kernel("log", -1.0 / (2.0 * math.pi))


def test_step_function_properties():
    t = np.linspace(-0.5, 1.5, 401)
    s = smoothing.step(t)
    assert np.all(s[t <= 0] == 1.0) and np.all(s[t >= 1] == 0.0)
    assert np.all(np.diff(s) <= 1e-15)                     # non-increasing
    # C-infinity at the ends: flat to all orders (tiny derivatives next to 0 and 1)
    assert 1.0 - smoothing.step(np.array([1e-3]))[0] < 1e-300
    assert smoothing.step(np.array([1 - 1e-3]))[0] < 1e-300


@pytest.mark.parametrize("k", [(0, 0), (1, 0), (3, -2), (-5, 7)])
def test_chihat_disc_against_quadrature(k):
    n, b, R, c = 8, 2, 0.3, (0.5, 0.5)
    tab = smoothing.chihat_disc(n, b, c, R)
    nb = n * b
    got = tab[k[0] % nb, k[1] % nb]
    f = lambda r, th: np.exp(-2j * math.pi * (k[0] * (c[0] + r * math.cos(th))
                                                + k[1] * (c[1] + r * math.sin(th))) / b) * r
    re = integrate.dblquad(lambda r, th: f(r, th).real, 0, 2 * math.pi, 0, R, epsabs=1e-13)[0]
    im = integrate.dblquad(lambda r, th: f(r, th).imag, 0, 2 * math.pi, 0, R, epsabs=1e-13)[0]
    assert abs(got - (re + 1j * im) / b ** 2) < 1e-11


def test_chihat_square_against_quadrature():
    n, b = 6, 3
    tab = smoothing.chihat_square(n, b, 0.3, 0.7)
    nb = n * b
    for k in [(0, 0), (2, -1), (-4, 5)]:
        one = lambda kk: integrate.quad(lambda y: math.cos(2 * math.pi * kk * y / b), 0.3, 0.7)[0] \
            - 1j * integrate.quad(lambda y: math.sin(2 * math.pi * kk * y / b), 0.3, 0.7)[0]
        assert abs(tab[k[0] % nb, k[1] % nb] - one(k[0]) * one(k[1]) / b ** 2) < 1e-13


def test_series_on_grid_bruteforce():
    n, b = 8, 2
    coef = smoothing.chihat_disc(n, b, (0.5, 0.5), 0.3)
    got = smoothing.series_on_grid(coef, n, b)
    k = moments.frequencies(n * b)
    for j in [(0, 0), (4, 4), (7, 1)]:
        ph = np.exp(2j * math.pi * (k[:, None] * j[0] + k[None, :] * j[1]) / (n * b))
        assert abs(got[j] - np.sum(coef * ph)) < 1e-14
    # Exactly real for a disc centred at (0.5, 0.5) with n divisible by 4.
    assert np.max(np.abs(got.imag)) < 1e-15


def test_fourier_smoothing_second_order_disc():
    # Section 2.4 / Table conv_FS: with smoothing the error decays at second order
    # (noc -> 2); without it, at first order.  Exact: the disc's log potential.
    R = 0.25
    fs, wfs = [], []
    for n in (32, 64, 128, 256):
        exact = cf.disc_log_potential(R, synth.radius(n))
        g = moments.ghat_table(LAPLACE, n, B, A2)
        u_fs = smoothing.smoothed_disc_density(n, B, R)
        fs.append(metrics.rel_linf(np.real(scheme.apply(u_fs, g, B)), exact))
        u_plain = (synth.radius(n) <= R).astype(float)
        wfs.append(metrics.rel_linf(np.real(scheme.apply(u_plain, g, B)), exact))
    rates_fs = [metrics.noc(fs[i], fs[i + 1]) for i in range(3)]
    # Table conv_FS itself shows 2.42, 2.57, 2.07, 2.04 before settling at 2.
    assert all(1.7 < r < 2.7 for r in rates_fs), rates_fs
    assert abs(rates_fs[-1] - 2.0) < 0.2
    assert fs[-1] < wfs[-1] / 20


def test_ls_gmres_matches_dense_solve():
    kappa = 20.0
    for n in (8, 16):
        g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A2)
        m = synth.contrast(n)
        ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(3020))
        xd = ls.dense_solve(m, ui, g, B, kappa)
        xg, info = ls.gmres(m, ui, g, B, kappa, tol=1e-13, restart=20)
        assert info["converged"]
        assert metrics.rel_linf(xg, xd) < 1e-11
        res = ui - ls.matvec(xg, m, g, B, kappa)
        assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1e-13


def test_ls_zero_contrast_returns_incident_field():
    n, kappa = 16, 40.0
    g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A2)
    ui = synth.plane_wave(n, kappa, 0.7)
    x, info = ls.gmres(np.zeros((n, n)), ui, g, B, kappa, tol=1e-12)
    assert np.max(np.abs(x - ui)) < 1e-14 and info["matvecs"] <= 2


def test_ls_solution_satisfies_helmholtz_structure():
    # The scattered field u - u_inc equals -kappa^2 A_n(m u) by construction.
    n, kappa = 16, 20.0
    g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A2)
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, 1.1)
    x, _ = ls.gmres(m, ui, g, B, kappa, tol=1e-13)
    sc = x - ui
    assert metrics.rel_linf(sc, -kappa ** 2 * scheme.apply(m * x, g, B)) < 1e-10
