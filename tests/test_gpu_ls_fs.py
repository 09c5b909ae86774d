"""Fourier smoothing inside the Lippmann-Schwinger solver (Section 2.4 applied
to the density m u of Section 3.3; Example 9, Table Scat_FS) through the
C-ABI (ls_solve_fs), against the CPU oracle.

The contrast m = m_tilde on a disc or square Omega and 0 outside has a jump
across the boundary of Omega; the operator uses m_s = m_tilde chi^n_Omega psi.
Parity: the GPU solution against the oracle's dense solve with the oracle's
own m_s (smoothing.smoothed_*_density), relative L-infinity <= 1e-10.
Property: with smoothing the solution converges at second order (Table
Scat_FS reports noc -> 2), and far faster than with the sampled indicator.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ls as ols
from oracle import metrics, smoothing
from tests.gpu_common import B, oracle_table, plan_kwargs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

R_DISC = 0.25          # disc radius (the paper does not give its own): kappa R = 5 at kappa = 20
PSI_R2 = 0.39


@pytest.fixture(scope="module")
def api():
    from paper_2107_03958_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _api


def _gpu(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def _disc(api, radius=R_DISC):
    return api.FsDesc("disc", 0.5, 0.5, radius, radius, PSI_R2)


@pytest.mark.parametrize("n", [32, 64])
@pytest.mark.parametrize("varying", [False, True])
def test_ls_fs_disc_vs_dense(api, n, varying):
    kappa = 20.0
    mt = -np.ones((n, n)) if not varying else -(1.0 + 0.5 * synth.cutoff(n))
    ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(synth.SEED_LS_ANGLE + 20))
    plan = api.ConvPlan(n=n, **plan_kwargs("helm20"))
    u, info = plan.ls_solve(_gpu(mt, torch.float64), _gpu(ui, torch.complex128), tol=1e-12, restart=40,
                            fs=_disc(api))
    assert info.status == 0, info
    ms = smoothing.smoothed_disc_density(n, B, R_DISC, r2=PSI_R2, u_tilde=mt)
    g = oracle_table("helm20", n)
    ref = ols.dense_solve(ms, ui, g, B, kappa)
    got = u.cpu().numpy()
    assert metrics.rel_linf(got, ref) <= 1e-10
    res = ui - ols.matvec(got, ms, g, B, kappa)
    assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1e-11


def test_ls_fs_square_vs_dense(api):
    n, kappa, h = 64, 20.0, 0.2
    mt = -np.ones((n, n))
    ui = synth.plane_wave(n, kappa, 0.7)
    plan = api.ConvPlan(n=n, **plan_kwargs("helm20"))
    fs = api.FsDesc("square", 0.5, 0.5, h, h * math.sqrt(2), PSI_R2)
    u, info = plan.ls_solve(_gpu(mt, torch.float64), _gpu(ui, torch.complex128), tol=1e-12, restart=40, fs=fs)
    assert info.status == 0, info
    ms = smoothing.smoothed_square_density(n, B, 0.5 - h, 0.5 + h, h * math.sqrt(2), PSI_R2, u_tilde=mt)
    ref = ols.dense_solve(ms, ui, oracle_table("helm20", n), B, kappa)
    assert metrics.rel_linf(u.cpu().numpy(), ref) <= 1e-10


def test_ls_fs_mixed_precision(api):
    n, kappa = 64, 20.0
    mt = -np.ones((n, n))
    ui = synth.plane_wave(n, kappa, 0.4)
    plan = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("helm20"))
    u, info = plan.ls_solve(_gpu(mt, torch.float64), _gpu(ui, torch.complex128), tol=1e-8, restart=30,
                            mixed=True, fs=_disc(api))
    assert info.status == 0, info
    ms = smoothing.smoothed_disc_density(n, B, R_DISC, r2=PSI_R2, u_tilde=mt)
    res = ui - ols.matvec(u.cpu().numpy(), ms, oracle_table("helm20", n), B, kappa)
    assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1.2e-8


def _solve(api, n, kappa, contrast, fs):
    plan = api.ConvPlan(n=n, **plan_kwargs("helm20"))
    ui = synth.plane_wave(n, kappa, 0.0)
    u, info = plan.ls_solve(_gpu(contrast, torch.float64), _gpu(ui, torch.complex128), tol=1e-11, restart=50,
                            fs=fs)
    assert info.status == 0, info
    return u.cpu().numpy()


def test_ls_fs_second_order(api):
    # Convergence study in the manner of Table Scat_FS (disc, m = -1 inside):
    # errors at the points of the coarse grid against a smoothed solve at n = 1024.
    kappa, nref = 20.0, 1024
    ref = _solve(api, nref, kappa, -np.ones((nref, nref)), _disc(api))
    fs_err, plain_err = [], []
    for n in (64, 128, 256):
        step = nref // n
        r = ref[::step, ::step]
        u_fs = _solve(api, n, kappa, -np.ones((n, n)), _disc(api))
        fs_err.append(metrics.rel_linf(u_fs, r))
        indicator = -(synth.radius(n) < R_DISC).astype(np.float64)
        u_plain = _solve(api, n, kappa, indicator, None)
        plain_err.append(metrics.rel_linf(u_plain, r))
    noc = [math.log2(fs_err[i] / fs_err[i + 1]) for i in range(len(fs_err) - 1)]
    assert min(noc) >= 1.5 and np.mean(noc) >= 1.7, (fs_err, noc)
    assert fs_err[-1] * 3.0 <= plain_err[-1], (fs_err, plain_err)


def test_ls_fs_rejects(api):
    from paper_2107_03958_amd import _lib as L
    n = 32
    plan = api.ConvPlan(n=n, **plan_kwargs("helm20"))
    m = _gpu(-np.ones((n, n)), torch.float64)
    ui = _gpu(synth.plane_wave(n, 20.0, 0.0), torch.complex128)
    with pytest.raises(L.WsError) as e:
        plan.ls_solve(m, ui, fs=api.FsDesc("none", 0.5, 0.5, 0.2, 0.2, 0.39))
    assert e.value.code == L.WS_EINVAL
    with pytest.raises(L.WsError) as e:
        plan.ls_solve(m, ui, fs=api.FsDesc("disc", 0.51, 0.5, 0.2, 0.2, 0.39))   # centre off the grid
    assert e.value.code == L.WS_EUNSUPPORTED
    p3 = api.ConvPlan(n=n, b=3, **plan_kwargs("helm20"))
    with pytest.raises(L.WsError) as e:
        p3.ls_solve(m, ui, fs=_disc(api))
    assert e.value.code == L.WS_EUNSUPPORTED
