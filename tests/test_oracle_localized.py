"""Pins of the oracle's localised moments and Yukawa kernel (oracle/localized.py)."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import synth
from oracle import localized as lo
from oracle import moments, scheme

HERE = os.path.dirname(os.path.abspath(__file__))
B3 = 3
A3 = (B3 + math.sqrt(2) / 2 - 0.5) / 2


def _step_mp(t):
    if t <= 0:
        return mp.mpf(1)
    if t >= 1:
        return mp.mpf(0)
    return mp.exp(2 * mp.exp(-1 / t) / (t - 1))


@pytest.mark.parametrize("family", ["log", "power", "yukawa"])
def test_ghat_eta_against_mpmath(family):
    # the trapezoidal rule in tau after rho = beta tau^4 against 30-digit quadrature
    mp.mp.dps = 30
    beta, b, n = 0.25, 2, 64
    g = {"log": np.log, "power": lambda r: r ** -0.5, "yukawa": lambda r: lo.yukawa(r, 20.0)}[family]
    gm = {"log": mp.log, "power": lambda r: r ** mp.mpf(-0.5), "yukawa": lambda r: mp.besselk(0, 20 * r)}[family]
    ks = np.array([0.0, 1.0, 7.5, 40.0, 90.0])
    got = lo.ghat_eta(g, ks, beta, b, 4, lo.nodes(n, beta))
    for k, v in zip(ks, got):
        xi = 2 * mp.pi * k / b
        f = lambda r: gm(r) * _step_mp((r - beta / 2) / (beta / 2)) * mp.besselj(0, xi * r) * r
        pts = [0, beta / 2] + [beta / 2 + (beta / 2) * i / 8 for i in range(1, 9)]
        ref = 2 * mp.pi * mp.quad(f, pts)
        assert abs(v - float(ref)) <= 1e-13 * abs(got[0]), (family, k)


@pytest.mark.parametrize("kappa", [1.0, 200.0])
def test_yukawa_closed_form_against_mpmath(kappa):
    mp.mp.dps = 30
    a, b = A3, B3
    ks = np.array([0.0, 1.0, 5.0, 33.0])
    got = lo.yukawa_global(ks, a, b, kappa)
    for k, v in zip(ks, got):
        xi = 2 * mp.pi * k / b
        f = lambda r: r * mp.besselk(0, kappa * r) * mp.besselj(0, xi * r)
        pts = [0] + [a * i / 16 for i in range(1, 17)]
        ref = 2 * mp.pi * mp.quad(f, pts)
        assert abs(v - float(ref)) <= 1e-13 * max(abs(float(ref)), abs(got[0])), (kappa, k)


def _yukawa_case(n, kappa, delta):
    x1, x2 = synth.grid(n)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2
    f = ((-4.0 * r2 + 4.0 * delta ** 2) / delta ** 4 + kappa ** 2) * np.exp(-r2 / delta ** 2)
    return f, np.exp(-r2 / delta ** 2)


def test_table_yukawa():
    # the global scheme with the closed-form truncated Yukawa moments reproduces
    # the paper's printed errors (tests/golden/table_yukawa.json)
    gold = json.load(open(os.path.join(HERE, "golden", "table_yukawa.json")))
    delta = gold["delta"]
    for kap_s, rows in gold["eps"].items():
        kappa = float(kap_s)
        for n_s, printed in rows.items():
            n = int(n_s)
            f, exact = _yukawa_case(n, kappa, delta)
            t = lo.yukawa_global_table(n, B3, A3, kappa, 1.0 / (2.0 * math.pi))
            eps = np.max(np.abs(np.real(scheme.apply(f, t, B3)) - exact)) / np.max(exact)
            if printed > 1e-14:
                assert printed / 2.0 <= eps <= printed * 2.0, (kappa, n, eps, printed)
            else:
                assert eps <= 1e-14, (kappa, n, eps)          # at the rounding level


def test_localised_equals_global_log_conv1_loc():
    # Table Conv1_loc's claim: the localised scheme is as accurate as the global
    # one (log kernel, u = (x1(1-x1)x2(1-x2))^3, b = 3), errors against the
    # global scheme at n = 256
    kern = moments.Kernel("log", 1.0)

    def dens(n):
        x1, x2 = synth.grid(n)
        return (x1 * (1 - x1) * x2 * (1 - x2)) ** 3

    nref = 256
    ref = np.real(scheme.apply(dens(nref), moments.ghat_table(kern, nref, B3, A3), B3))
    for n in (32, 64):
        r = ref[:: nref // n, :: nref // n]
        gl = np.real(scheme.apply(dens(n), moments.ghat_table(kern, n, B3, A3), B3))
        loc = np.real(scheme.apply(dens(n), lo.ghat_table_local(np.log, n, B3, 1.0), B3))
        eg = np.max(np.abs(gl - r)) / np.max(np.abs(r))
        el = np.max(np.abs(loc - r)) / np.max(np.abs(r))
        assert el <= 1.5 * eg and eg <= 1.5 * el, (n, eg, el)


def test_localised_yukawa_against_closed_form():
    # with a wide window the localised Yukawa table gives the closed-form scheme's result
    n, kappa = 64, 1.0
    f, _ = _yukawa_case(n, kappa, 0.08)
    sc = 1.0 / (2.0 * math.pi)
    glob = np.real(scheme.apply(f, lo.yukawa_global_table(n, B3, A3, kappa, sc), B3))
    loc = np.real(scheme.apply(f, lo.ghat_table_local(lambda r: lo.yukawa(r, kappa, sc), n, B3, 1.5), B3))
    assert np.max(np.abs(loc - glob)) <= 1e-12 * np.max(np.abs(glob))


def test_khat_smooth_is_the_trapezoid_sum():
    # Khat through the table equals the trapezoidal sum h^2 sum_j g_s(x_i - x_j) u_j, term by term
    n, b, beta = 12, 2, 0.4
    g = lambda r: lo.yukawa(r, 3.0)
    rng = np.random.default_rng(4)
    u = rng.normal(size=(n, n))
    t = np.real(scheme.apply(u, lo.khat_smooth(g, n, b, beta), b))
    h = 1.0 / n
    for i1, i2 in [(0, 0), (5, 7), (11, 3)]:
        d1 = (i1 - np.arange(n))[:, None] * h
        d2 = (i2 - np.arange(n))[None, :] * h
        r = np.hypot(d1, d2)
        gs = np.zeros_like(r)
        nz = r > 0
        gs[nz] = g(r[nz]) * (1.0 - lo.eta(r[nz], beta))
        assert abs(t[i1, i2] - h * h * np.sum(gs * u)) <= 1e-13 * np.max(np.abs(t))
