"""The Yukawa kernel and localised moments (Section 2.3) on the GPU, against
the oracle (oracle/localized.py, pinned by 30-digit quadrature and by the
paper's Table yukawa, tests/golden/table_yukawa.json), through the C-ABI.

Bar: FP64 relative L-infinity <= 1e-12 (applies), moments <= 1e-13 of the
largest; FP32 <= 2e-6.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import localized as lo
from oracle import metrics, scheme

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
SC = 1.0 / (2.0 * math.pi)


def _a(b):
    return (b + math.sqrt(2) / 2 - 0.5) / 2


@pytest.fixture(scope="module")
def api():
    from paper_2107_03958_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _api


def _gpu(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def _g(family, kappa=1.0, gamma=-0.5):
    return {"log": np.log, "power": lambda r: r ** gamma,
            "yukawa": lambda r: lo.yukawa(r, kappa)}[family]


@pytest.mark.parametrize("b", [2, 3])
@pytest.mark.parametrize("kappa", [1.0, 200.0])
@pytest.mark.parametrize("n", [16, 64, 256])
def test_yukawa_global_apply(api, b, kappa, n):
    u = synth.smooth_density(n, 1200 + n)
    plan = api.ConvPlan("yukawa", n=n, b=b, kappa=kappa, scale=SC)
    got = plan.apply(_gpu(u[None]))[0].cpu().numpy()
    ref = np.real(scheme.apply(u, lo.yukawa_global_table(n, b, _a(b), kappa, SC), b))
    assert metrics.rel_linf(got, ref) <= 1e-12


def test_yukawa_fp32(api):
    n, kappa = 128, 20.0
    u = synth.smooth_density(n, 77)
    plan = api.ConvPlan("yukawa", n=n, kappa=kappa, scale=SC, precision="fp32")
    got = plan.apply(_gpu(u[None], torch.float32))[0].double().cpu().numpy()
    ref = np.real(scheme.apply(u, lo.yukawa_global_table(n, 2, _a(2), kappa, SC), 2))
    assert metrics.rel_linf(got, ref) <= 2e-6


def test_table_yukawa_on_gpu(api):
    gold = json.load(open(os.path.join(HERE, "golden", "table_yukawa.json")))
    d = gold["delta"]
    for kap_s, rows in gold["eps"].items():
        kappa = float(kap_s)
        for n_s, printed in rows.items():
            n = int(n_s)
            x1, x2 = synth.grid(n)
            r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2
            f = ((-4.0 * r2 + 4.0 * d * d) / d ** 4 + kappa ** 2) * np.exp(-r2 / d ** 2)
            exact = np.exp(-r2 / d ** 2)
            plan = api.ConvPlan("yukawa", n=n, b=3, kappa=kappa, scale=SC)
            got = plan.apply(_gpu(f[None]))[0].cpu().numpy()
            eps = np.max(np.abs(got - exact)) / np.max(exact)
            if printed > 1e-14:
                assert printed / 2.0 <= eps <= printed * 2.0, (kappa, n, eps, printed)
            else:
                assert eps <= 1e-14, (kappa, n, eps)


@pytest.mark.parametrize("family,b,n,beta", [("log", 2, 32, 0.5), ("power", 2, 64, 0.25), ("yukawa", 3, 32, 1.0),
                                             ("log", 3, 64, 1.0), ("yukawa", 2, 128, 0.25)])
def test_localised_apply_and_moments(api, family, b, n, beta):
    kappa = 5.0
    g = _g(family, kappa)
    kw = dict(kappa=kappa) if family == "yukawa" else dict(gamma=-0.5) if family == "power" else {}
    plan = api.ConvPlan(family, n=n, b=b, beta=beta, **kw)
    table = lo.ghat_table_local(g, n, b, beta)
    u = synth.full_support_density(n, 5100) if b == 3 else synth.smooth_density(n, 5100)
    got = plan.apply(_gpu(u[None]))[0].cpu().numpy()
    ref = np.real(scheme.apply(u, table, b))
    assert metrics.rel_linf(got, ref) <= 1e-12
    nb = n * b
    rng = np.random.default_rng(n)
    k1 = np.concatenate([[0, 1, -nb // 2, nb // 2 - 1], rng.integers(-nb // 2, nb // 2, 30)])
    k2 = np.concatenate([[0, 0, -nb // 2, 3], rng.integers(-nb // 2, nb // 2, 30)])
    mom = plan.moments(k1, k2)
    refm = table[k1 % nb, k2 % nb]
    assert np.max(np.abs(mom - refm)) <= 1e-13 * np.max(np.abs(table))


def test_localised_large_plan_builds(api):
    # n = 2048 with beta = 32 h: the O(n^2)-cost construction the localisation is for
    n = 2048
    plan = api.ConvPlan("log", n=n, beta=32.0 / n)
    g = lo.ghat_eta(np.log, np.array([0.0, 100.0, 1000.0]), 32.0 / n, 2.0, 4, lo.nodes(n, 32.0 / n))
    mom = plan.moments(np.array([0, 100, 1000]), np.array([0, 0, 0]))
    # Khat adds the smooth part; at k = 0 it is the trapezoid sum of g (1 - eta) over (-n, n)^2
    h = 1.0 / n
    m = np.arange(n, dtype=np.float64)
    r = h * np.hypot(m[:, None], m[None, :])
    w = np.where(m == 0, 1.0, 2.0)
    gs = np.zeros_like(r)
    nz = r > 0
    gs[nz] = np.log(r[nz]) * (1.0 - lo.eta(r[nz], 32.0 / n))
    k0 = g[0] + h * h * np.sum(np.outer(w, w) * gs)
    assert abs(mom[0] - k0) <= 1e-12 * abs(k0)
    assert np.all(np.isfinite(mom))


def test_localised_rejects(api):
    from paper_2107_03958_amd import _lib as L
    with pytest.raises(L.WsError) as e:
        api.ConvPlan("log", n=64, beta=2.0)                    # beyond a
    assert e.value.code == L.WS_EINVAL
    with pytest.raises(L.WsError) as e:
        api.ConvPlan("helmholtz", n=64, kappa=20.0, beta=0.1)
    assert e.value.code == L.WS_EUNSUPPORTED
    with pytest.raises(L.WsError) as e:
        api.ConvPlan("log", n=2048, beta=1.0)                  # too many quadrature nodes
    assert e.value.code == L.WS_EUNSUPPORTED
    with pytest.raises(L.WsError) as e:
        api.ConvPlan("yukawa", n=64, kappa=0.0)
    assert e.value.code == L.WS_EINVAL
