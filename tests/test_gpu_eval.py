"""Evaluation of A_n u at arbitrary points (conv_eval; Section 2.1, eq. An read
at any x, equivalently eqs. quad / quad_wts) through the C-ABI, against the
oracle's scheme.apply_at (pinned against the brute-force quadrature weights).

Bar: relative (to the largest |value|) error <= 1e-12 in FP64.
"""
import math

import numpy as np
import pytest

import synth
from oracle import moments, scheme
from tests.gpu_common import A_DEFAULT, B, oracle_kernel, oracle_table, plan_kwargs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = 1e-12


@pytest.fixture(scope="module")
def api():
    from paper_2107_03958_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _api


def _targets(count, seed):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(count, 2))
    # a few outside D (the series is b-periodic) and on its corners
    extra = np.array([[0.0, 0.0], [1.0, 1.0], [-0.25, 0.5], [1.3, 2.7], [0.5, -1.1]])
    return np.concatenate([pts, extra])


def _density(kname, n, seed):
    u = synth.smooth_density(n, seed)
    if kname.startswith("helm"):
        rng = np.random.default_rng(seed)
        u = u * (1.0 + 1j * rng.normal(size=(n, n)))
    return u


@pytest.mark.parametrize("kname", ["log", "pow-1/2", "helm20"])
@pytest.mark.parametrize("n", [16, 64, 128])
def test_eval_off_grid_vs_oracle(api, kname, n):
    u = _density(kname, n, 1000 + n)
    pts = _targets(40, n)
    plan = api.ConvPlan(n=n, **plan_kwargs(kname))
    dt = torch.complex128 if kname.startswith("helm") else torch.float64
    got = plan.eval(torch.as_tensor(u).to(dt).cuda(), torch.as_tensor(pts).cuda()).cpu().numpy()
    ref = scheme.apply_at(u, oracle_table(kname, n), B, pts)
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref)), (kname, n)


def test_eval_period3_vs_oracle(api):
    n, b = 64, 3
    a3 = (b + math.sqrt(2) / 2 - 0.5) / 2
    u = synth.full_support_density(n, synth.SEED_FULL_SUPPORT)
    pts = _targets(30, 7)
    plan = api.ConvPlan(n=n, b=b, **plan_kwargs("log"))
    got = plan.eval(torch.as_tensor(u).cuda(), torch.as_tensor(pts).cuda()).cpu().numpy()
    g = moments.ghat_table(oracle_kernel("log"), n, b, a3)
    ref = scheme.apply_at(u, g, b, pts)
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref))


def test_eval_on_grid_equals_apply(api):
    n = 256
    u = synth.smooth_density(n, 21)
    plan = api.ConvPlan(n=n, **plan_kwargs("pow-1/3"))
    ut = torch.as_tensor(u).cuda()
    full = plan.apply(ut[None].clone())[0].cpu().numpy()
    rng = np.random.default_rng(5)
    idx = rng.integers(0, n, size=(64, 2))
    pts = idx.astype(np.float64) / n
    got = plan.eval(ut, torch.as_tensor(pts).cuda()).cpu().numpy()
    ref = full[idx[:, 0], idx[:, 1]]
    scale = np.max(np.abs(full))
    assert np.max(np.abs(got.real - ref)) <= TOL * scale
    assert np.max(np.abs(got.imag)) <= TOL * scale


def test_eval_large_grid_sampled(api):
    n = 512
    u = synth.smooth_density(n, 33)
    pts = _targets(16, 11)
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    got = plan.eval(torch.as_tensor(u).cuda(), torch.as_tensor(pts).cuda()).cpu().numpy()
    ref = scheme.apply_at(u, oracle_table("log", n), B, pts)
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref))


@pytest.mark.slow
def test_eval_n2048_sampled(api):
    # the spectrum pass's column tiles at the largest grid (split exchange)
    n = 2048
    u = synth.smooth_density(n, 34)
    pts = _targets(6, 13)
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    got = plan.eval(torch.as_tensor(u).cuda(), torch.as_tensor(pts).cuda()).cpu().numpy()
    ref = scheme.apply_at(u, oracle_table("log", n), B, pts)
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref))


@pytest.mark.slow
def test_eval_period3_n2048(api):
    # period 3 at the largest grid (6144^2 spectrum, split-exchange column tiles): off-grid targets
    # against the oracle, on-grid targets against conv_apply (itself checked against the oracle there)
    n, b = 2048, 3
    a3 = (b + math.sqrt(2) / 2 - 0.5) / 2
    u = synth.full_support_density(n, synth.SEED_FULL_SUPPORT + 5)
    ut = torch.as_tensor(u).cuda()
    plan = api.ConvPlan(n=n, b=b, **plan_kwargs("log"))
    pts = _targets(4, 17)
    got = plan.eval(ut, torch.as_tensor(pts).cuda()).cpu().numpy()
    ref = scheme.apply_at(u, moments.ghat_table(oracle_kernel("log"), n, b, a3), b, pts)
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref))
    full = plan.apply(ut[None].clone())[0].cpu().numpy()
    idx = np.random.default_rng(6).integers(0, n, size=(32, 2))
    on = plan.eval(ut, torch.as_tensor(idx.astype(np.float64) / n).cuda()).cpu().numpy()
    scale = np.max(np.abs(full))
    assert np.max(np.abs(on.real - full[idx[:, 0], idx[:, 1]])) <= TOL * scale
    assert np.max(np.abs(on.imag)) <= TOL * scale


def test_eval_target_tiles(api):
    # more targets than one tile of the matrix product (4096 at this size): a full tile and a
    # ragged one of 4, against the oracle
    n = 64
    u = synth.smooth_density(n, 41)
    pts = _targets(4100, 23)
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    got = plan.eval(torch.as_tensor(u).cuda(), torch.as_tensor(pts).cuda()).cpu().numpy()
    ref = scheme.apply_at(u, oracle_table("log", n), B, pts)
    assert np.max(np.abs(got - ref)) <= TOL * np.max(np.abs(ref))


def test_eval_edge_cases(api):
    from paper_2107_03958_amd import _lib as L
    n = 32
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    u = torch.as_tensor(synth.smooth_density(n, 2)).cuda()
    empty = plan.eval(u, torch.zeros((0, 2), dtype=torch.float64, device="cuda"))
    assert empty.numel() == 0
    one = plan.eval(u, torch.tensor([[0.3, 0.6]], dtype=torch.float64, device="cuda")).cpu().numpy()
    ref = scheme.apply_at(synth.smooth_density(n, 2), oracle_table("log", n), B, np.array([[0.3, 0.6]]))
    assert abs(one[0] - ref[0]) <= TOL * abs(ref[0])
    p32 = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("log"))
    with pytest.raises(L.WsError) as e:
        p32.eval(u.float(), torch.zeros((1, 2), dtype=torch.float64, device="cuda"))
    assert e.value.code == L.WS_EUNSUPPORTED
