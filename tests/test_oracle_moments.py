"""Pins of the oracle's kernel moments (oracle/moments.py) against high-precision quadrature.

The defining integral (Section 2.2, eq. ghat) is evaluated with mpmath at 30
digits, split at every half period of J0 so the oscillatory integrand is
resolved; the power-kernel closed form with Lommel functions (Section 2.2)
is evaluated from the definition of S_{mu,nu} (DLMF 11.9); gamma = -1 is also checked against the
Struve-function closed form.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

from oracle import moments

B = 2
A = (B + math.sqrt(2) / 2 - 0.5) / 2     # default truncation radius for b = 2


def _mp_radial(f, xi, a, power=None):
    """2 pi int_0^a f(rho) J0(xi rho) rho d rho in mpmath (30 digits).

    The substitution rho = t^2 removes the endpoint singularity of weakly
    singular integrands; the t-interval is split at every half period of J0.
    """
    with mp.workdps(30):
        npts = max(2, int(math.ceil(float(xi) * a / math.pi)) + 1)
        pts = [mp.sqrt(mp.mpf(a) * i / npts) for i in range(npts + 1)]
        val = mp.quad(lambda t: f(t * t) * mp.besselj(0, xi * t * t) * t * t * 2 * t, pts)
        return complex(2 * mp.pi * val)


@pytest.mark.parametrize("k", [0, 1, 7, 40])
def test_log_closed_form_vs_quadrature(k):
    xi = 2 * math.pi * k / B
    ref = _mp_radial(lambda r: -mp.log(r) / (2 * mp.pi), xi, A).real
    got = moments.log_paper(np.array([float(k)]), A, B)[0]
    assert abs(got - ref) <= 1e-15 * max(1.0, abs(ref))


@pytest.mark.parametrize("kappa,k", [(20.0, 0), (20.0, 3), (20.0, 11), (40.0, 0), (40.0, 17)])
def test_helmholtz_closed_form_vs_quadrature(kappa, k):
    xi = 2 * math.pi * k / B
    ref = _mp_radial(lambda r: 0.25j * mp.hankel1(0, kappa * r), xi, A)
    got = moments.helmholtz_paper(np.array([float(k)]), A, B, kappa)[0]
    assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref))


def test_helmholtz_printed_k0_sign_disagrees():
    # The |k| = 0 line as printed (+2/(kappa pi)) is off by exactly 2/kappa^2;
    # the oracle uses -2/(kappa pi), the k -> 0 limit of the generic line.
    kappa = 20.0
    ka = kappa * A
    printed = math.pi / (2 * kappa) * (1j * A * special.j1(ka) - A * special.y1(ka) + 2 / (kappa * math.pi))
    got = moments.helmholtz_paper(np.array([0.0]), A, B, kappa)[0]
    assert abs((printed - got) - 2 / kappa ** 2) < 1e-15
    near = moments.helmholtz_paper(np.array([1e-7]), A, B, kappa)[0]
    assert abs(near - got) < 1e-10


def test_helmholtz_resonance_line():
    # kappa = 5 pi puts |k| = 5 exactly on the resonance xi = kappa (b = 2).
    kappa = 5 * math.pi
    ref = _mp_radial(lambda r: 0.25j * mp.hankel1(0, kappa * r), kappa, A)
    got = moments.helmholtz_paper(np.array([5.0]), A, B, kappa)[0]
    assert abs(got - ref) <= 1e-14 * abs(ref)
    # Just off resonance the generic line (0/0-like) still matches quadrature.
    xi_off = math.pi * (5.0 + 1e-5)
    ref_off = _mp_radial(lambda r: 0.25j * mp.hankel1(0, kappa * r), xi_off, A)
    off = moments.helmholtz_paper(np.array([5.0 + 1e-5]), A, B, kappa)[0]
    assert abs(off - ref_off) < 1e-9 * abs(ref_off)


@pytest.mark.parametrize("gamma", [-0.5, -1.0 / 3.0, -1.0, -1.5])
@pytest.mark.parametrize("k", [1, 9, 40])
def test_power_quadrature_vs_mpmath(gamma, k):
    xi = 2 * math.pi * k / B
    ref = _mp_radial(lambda r: r ** gamma, xi, A).real
    got = moments.ghat(moments.Kernel("power", 1.0, gamma), np.array([float(k)]), A, B)[0]
    assert abs(got - ref) <= 2e-14 * max(1.0, abs(ref))


def _lommel_S(mu, nu, z):
    """Lommel function S_{mu,nu}(z) from its definition through s_{mu,nu} (DLMF 11.9.3, 11.9.5)."""
    s_small = z ** (mu + 1) / ((mu + 1) ** 2 - nu ** 2) * mp.hyp1f2(
        1, (mu - nu + 3) / 2, (mu + nu + 3) / 2, -z * z / 4)
    c = 2 ** (mu - 1) * mp.gamma((mu - nu + 1) / 2) * mp.gamma((mu + nu + 1) / 2)
    return s_small + c * (mp.sin((mu - nu) * mp.pi / 2) * mp.besselj(nu, z)
                          - mp.cos((mu - nu) * mp.pi / 2) * mp.bessely(nu, z))


@pytest.mark.parametrize("gamma", [-0.5, -1.0 / 3.0, -1.5])
@pytest.mark.parametrize("k", [1, 9])
def test_power_matches_paper_lommel_form(gamma, k):
    # Closed form for (1/2pi)|x|^gamma (Section 2.2) with Lommel functions S_{mu,nu}.
    with mp.workdps(40):
        g = mp.mpf(gamma)
        xi = 2 * mp.pi * k / B
        z = xi * A
        first = 2 ** (1 + g) / xi ** (2 + g) * mp.gamma(1 + g / 2) / mp.gamma(-g / 2)
        second = A / xi ** (1 + g) * (g * mp.besselj(0, z) * _lommel_S(g, mp.mpf(-1), z)
                                      + mp.besselj(1, z) * _lommel_S(1 + g, mp.mpf(0), z))
        paper = float(first + second)
    got = moments.power_radial(np.array([float(k)]), A, B, gamma)[0]
    assert abs(got - paper) <= 1e-14 * max(1.0, abs(paper))


@pytest.mark.parametrize("k", [0, 2, 13])
def test_power_gamma_minus_one_struve_form(k):
    # (2 pi |x|)^-1: ghat = a (J0 + pi/2 (J1 H0 - J0 H1)) with Struve H_nu (Section 2.2).
    z = 2 * math.pi * k * A / B
    if k == 0:
        paper = A
    else:
        paper = A * (special.j0(z) + math.pi / 2 * (special.j1(z) * special.struve(0, z)
                                                     - special.j0(z) * special.struve(1, z)))
    got = moments.power_radial(np.array([float(k)]), A, B, -1.0)[0]
    assert abs(got - paper) <= 1e-13


def test_table_layout_and_symmetry():
    n, b = 8, 2
    tab = moments.ghat_table(moments.Kernel("log", 1.0), n, b, A)
    nb = n * b
    assert tab.shape == (nb, nb)
    k = moments.frequencies(nb)
    assert k[nb // 2] == -nb // 2 and k[1] == 1 and k[-1] == -1
    assert np.array_equal(tab, tab.T)
    assert np.array_equal(tab[1:, :], tab[1:, :][::-1, :])        # k1 -> -k1
    direct = moments.ghat(moments.Kernel("log", 1.0), np.array([math.hypot(3, 5)]), A, b)[0]
    assert abs(tab[3, nb - 5] - direct) < 1e-16 * abs(direct) + 1e-300


def test_kernel_scaling():
    kabs = np.array([0.0, 1.0, 5.0])
    base = moments.log_paper(kabs, A, B)
    got = moments.ghat(moments.Kernel("log", -1 / (2 * math.pi)), kabs, A, B)
    assert np.allclose(got, base, rtol=1e-15, atol=0)
