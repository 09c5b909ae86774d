"""GPU path vs the CPU oracle, element by element, through the C-ABI.

Bar: FP64 relative L-infinity (eq. rel-err form) <= 1e-12; FP32 relative
L-infinity <= 2e-6 and relative L2 <= 5e-7 against the FP64 oracle.
"""
import math

import numpy as np
import pytest

import synth
from oracle import ls as ols
from oracle import metrics, moments, scheme, smoothing
from tests.gpu_common import A_DEFAULT, B, oracle_kernel, oracle_table, plan_kwargs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def api():
    from paper_2107_03958_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _api


def _gpu(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


def test_config0_single_apply(api):
    n = 64
    u = synth.bump_density(n)
    plan = api.ConvPlan(n=n, **plan_kwargs("laplace"))
    assert abs(plan.a - A_DEFAULT) < 1e-15
    got = plan.apply(_gpu(u, torch.float64)).cpu().numpy()
    ref = np.real(scheme.apply(u, oracle_table("laplace", n), B))
    assert metrics.rel_linf(got, ref) <= FP64_TOL


@pytest.mark.parametrize("kname", ["log", "pow-1/2", "pow-1/3"])
@pytest.mark.parametrize("n", [16, 32, 128, 256])
def test_real_apply_batch(api, kname, n):
    us = np.stack([synth.smooth_density(n, 1000 + i) for i in range(3)])
    plan = api.ConvPlan(n=n, **plan_kwargs(kname))
    got = plan.apply(_gpu(us, torch.float64)).cpu().numpy()
    g = oracle_table(kname, n)
    for i in range(3):
        ref = np.real(scheme.apply(us[i], g, B))
        assert metrics.rel_linf(got[i], ref) <= FP64_TOL, (kname, n, i)


@pytest.mark.parametrize("n", [512, 1024])
def test_real_apply_n512_log(api, n):
    us = np.stack([synth.smooth_density(n, 1000 + i) for i in range(2)])
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    got = plan.apply(_gpu(us, torch.float64)).cpu().numpy()
    g = oracle_table("log", n)
    for i in range(2):
        assert metrics.rel_linf(got[i], np.real(scheme.apply(us[i], g, B))) <= FP64_TOL


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_power_apply_n512_config1(api, precision):
    # The batched-apply workload's second kernel |x|^-1/2 at its larger grid (512^2, a
    # 1024^2 FFT): smooth densities and a Fourier-smoothed disc against the oracle.
    n = 512
    us = np.stack([synth.smooth_density(n, synth.SEED_SMOOTH_BATCH + i) for i in range(2)]
                  + [np.ones((n, n))])
    R = synth.disc_radius(synth.SEED_DISC_BATCH)
    fs = [None, None, api.FsDesc("disc", 0.5, 0.5, R, R, 0.39)]
    plan = api.ConvPlan(n=n, precision=precision, **plan_kwargs("pow-1/2"))
    dt = torch.float64 if precision == "fp64" else torch.float32
    got = plan.apply(_gpu(us, dt), fs=fs).cpu().numpy().astype(np.float64)
    g = oracle_table("pow-1/2", n)
    dens = [us[0], us[1], smoothing.smoothed_disc_density(n, B, R, r2=0.39)]
    for i in range(3):
        ref = np.real(scheme.apply(dens[i], g, B))
        if precision == "fp64":
            assert metrics.rel_linf(got[i], ref) <= FP64_TOL, i
        else:
            assert metrics.rel_linf(got[i], ref) <= 2e-6 and metrics.rel_l2(got[i], ref) <= 5e-7, i


@pytest.fixture(scope="module")
def full_size_case():
    """Four seeded smooth densities at the largest grid (2048^2, a 4096^2 FFT) and their oracle applies."""
    n = 2048
    us = np.stack([synth.smooth_density(n, synth.SEED_PRECISION + i) for i in range(4)])
    g = oracle_table("log", n)
    refs = [np.real(scheme.apply(us[i], g, B)) for i in range(4)]
    oracle_table.cache_clear()
    return n, us, refs


@pytest.mark.slow
def test_full_size_fp64_apply(api, full_size_case):
    # batch 4 runs as two chunks at this size (the tail chunk holds fewer densities)
    n, us, refs = full_size_case
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    assert plan.chunk < 4 and 4 % plan.chunk != 0
    got = plan.apply(_gpu(us, torch.float64)).cpu().numpy()
    for i in range(4):
        assert metrics.rel_linf(got[i], refs[i]) <= FP64_TOL, i


@pytest.mark.slow
def test_full_size_fp32_apply(api, full_size_case):
    n, us, refs = full_size_case
    plan = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("log"))
    got = plan.apply(_gpu(us, torch.float32)).cpu().numpy().astype(np.float64)
    for i in range(4):
        assert metrics.rel_linf(got[i], refs[i]) <= 2e-6, i
        assert metrics.rel_l2(got[i], refs[i]) <= 5e-7, i


@pytest.mark.parametrize("kname", ["pow-1/2", "pow-1/3"])
def test_full_size_moments_sampled(api, kname):
    # the apply machinery is shared by every real kernel; what differs per
    # kernel is the moment table, checked here at the full size
    n = 2048
    plan = api.ConvPlan(n=n, **plan_kwargs(kname))
    rng = np.random.default_rng(11)
    k1 = np.concatenate([[0, 1, -n, -n, n - 1, 1447, 2047], rng.integers(-n, n, 60)])
    k2 = np.concatenate([[0, 0, 0, -n, n - 1, 1448, -2048], rng.integers(-n, n, 60)])
    got = plan.moments(k1, k2)
    kabs = np.sqrt((k1.astype(np.int64) ** 2 + k2.astype(np.int64) ** 2).astype(np.float64))
    ref = moments.ghat(oracle_kernel(kname), kabs, A_DEFAULT, B)
    scale = abs(moments.ghat(oracle_kernel(kname), np.zeros(1), A_DEFAULT, B)[0])
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale


@pytest.mark.slow
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_complex_apply_n1024(api, precision):
    n = 1024
    rng = np.random.default_rng(n)
    v = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * synth.cutoff(n)
    plan = api.ConvPlan(n=n, precision=precision, **plan_kwargs("helm40"))
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    got = plan.apply(_gpu(v, dt)).cpu().numpy().astype(np.complex128)
    ref = scheme.apply(v, oracle_table("helm40", n), B)
    if precision == "fp64":
        assert metrics.rel_linf(got, ref) <= FP64_TOL
    else:
        assert metrics.rel_linf(got, ref) <= 2e-6
        assert metrics.rel_l2(got, ref) <= 5e-7


@pytest.mark.slow
def test_complex_apply_n2048_fp64(api):
    # at the largest grid the FP64 column tiles exchange one real component
    # at a time (complex path: Helmholtz moments, full-spectrum columns)
    n = 2048
    rng = np.random.default_rng(n)
    v = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * synth.cutoff(n)
    plan = api.ConvPlan(n=n, **plan_kwargs("helm40"))
    got = plan.apply(_gpu(v, torch.complex128)).cpu().numpy()
    ref = scheme.apply(v, oracle_table("helm40", n), B)
    oracle_table.cache_clear()
    assert metrics.rel_linf(got, ref) <= FP64_TOL


@pytest.mark.parametrize("kname", ["helm20", "helm40"])
@pytest.mark.parametrize("n", [16, 64, 128])
def test_complex_apply(api, kname, n):
    rng = np.random.default_rng(n)
    v = (rng.normal(size=(2, n, n)) + 1j * rng.normal(size=(2, n, n))) * synth.cutoff(n)
    plan = api.ConvPlan(n=n, **plan_kwargs(kname))
    got = plan.apply(_gpu(v, torch.complex128)).cpu().numpy()
    g = oracle_table(kname, n)
    for i in range(2):
        assert metrics.rel_linf(got[i], scheme.apply(v[i], g, B)) <= FP64_TOL


@pytest.mark.parametrize("kname", ["log", "pow-1/2", "pow-1/3", "helm20"])
def test_moments_sampled(api, kname):
    n = 128
    plan = api.ConvPlan(n=n, **plan_kwargs(kname))
    rng = np.random.default_rng(5)
    k1 = np.concatenate([[0, 1, 0, 3, -n, -n, n - 1], rng.integers(-n, n, 40)])
    k2 = np.concatenate([[0, 0, 1, 4, 0, -n, n - 1], rng.integers(-n, n, 40)])
    got = plan.moments(k1, k2)
    full = oracle_table(kname, n)
    nb = n * B
    ref = np.array([full[a % nb, b % nb] for a, b in zip(k1, k2)])
    scale = np.max(np.abs(full))
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale


@pytest.mark.parametrize("shape", ["disc", "square"])
@pytest.mark.parametrize("n", [64, 128])
def test_fourier_smoothing_apply(api, shape, n):
    R = 0.25
    plan = api.ConvPlan(n=n, **plan_kwargs("laplace"))
    ut = np.ones((n, n))
    if shape == "disc":
        fs = api.FsDesc("disc", 0.5, 0.5, R, R, 0.39)
        dens = smoothing.smoothed_disc_density(n, B, R, r2=0.39)
    else:
        h = 0.15
        fs = api.FsDesc("square", 0.5, 0.5, h, h * math.sqrt(2), 0.39)
        dens = smoothing.smoothed_square_density(n, B, 0.5 - h, 0.5 + h, h * math.sqrt(2), 0.39)
    got = plan.apply(_gpu(ut, torch.float64).unsqueeze(0), fs=[fs]).cpu().numpy()[0]
    ref = np.real(scheme.apply(dens, oracle_table("laplace", n), B))
    assert metrics.rel_linf(got, ref) <= FP64_TOL


@pytest.mark.slow
def test_fourier_smoothing_apply_n2048(api):
    # the smoothing pre-pass's column tiles at the largest grid (both lines per
    # thread; split exchange in FP64), FP64 and FP32, against one oracle result
    n, R = 2048, 0.25
    fs = api.FsDesc("disc", 0.5, 0.5, R, R, 0.39)
    dens = smoothing.smoothed_disc_density(n, B, R, r2=0.39)
    ref = np.real(scheme.apply(dens, oracle_table("laplace", n), B))
    oracle_table.cache_clear()
    plan = api.ConvPlan(n=n, **plan_kwargs("laplace"))
    got = plan.apply(_gpu(np.ones((n, n)), torch.float64).unsqueeze(0), fs=[fs]).cpu().numpy()[0]
    assert metrics.rel_linf(got, ref) <= FP64_TOL
    del plan
    p32 = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("laplace"))
    got32 = p32.apply(_gpu(np.ones((n, n)), torch.float32).unsqueeze(0), fs=[fs]).cpu().numpy()[0].astype(np.float64)
    assert metrics.rel_linf(got32, ref) <= 2e-6
    assert metrics.rel_l2(got32, ref) <= 5e-7


@pytest.mark.parametrize("n", [128, 1024])
def test_fourier_smoothing_apply_fp32(api, n):
    # the FP32 smoothing pre-pass (synthesised spectrum, FP32 column and row
    # transforms) against the FP64 oracle, to the FP32 bounds
    R = 0.25
    plan = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("laplace"))
    fs = api.FsDesc("disc", 0.5, 0.5, R, R, 0.39)
    dens = smoothing.smoothed_disc_density(n, B, R, r2=0.39)
    got = plan.apply(_gpu(np.ones((n, n)), torch.float32).unsqueeze(0), fs=[fs]).cpu().numpy()[0].astype(np.float64)
    ref = np.real(scheme.apply(dens, oracle_table("laplace", n), B))
    assert metrics.rel_linf(got, ref) <= 2e-6
    assert metrics.rel_l2(got, ref) <= 5e-7


def test_mixed_fs_and_plain_batch(api):
    n = 64
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    u0 = synth.smooth_density(n, 1003)
    R = synth.disc_radius(1100)
    us = np.stack([u0, np.ones((n, n))])
    fs = [None, api.FsDesc("disc", 0.5, 0.5, R, R, 0.39)]
    got = plan.apply(_gpu(us, torch.float64), fs=fs).cpu().numpy()
    g = oracle_table("log", n)
    assert metrics.rel_linf(got[0], np.real(scheme.apply(u0, g, B))) <= FP64_TOL
    dens = smoothing.smoothed_disc_density(n, B, R, r2=0.39)
    assert metrics.rel_linf(got[1], np.real(scheme.apply(dens, g, B))) <= FP64_TOL


@pytest.mark.parametrize("kname", ["log", "pow-1/2"])
@pytest.mark.parametrize("n", [16, 32, 64, 256])
def test_fp32_apply_bound(api, kname, n):
    us = np.stack([synth.smooth_density(n, 2000 + i) for i in range(2)])
    plan = api.ConvPlan(n=n, precision="fp32", **plan_kwargs(kname))
    got = plan.apply(_gpu(us, torch.float32)).cpu().numpy().astype(np.float64)
    g = oracle_table(kname, n)
    for i in range(2):
        ref = np.real(scheme.apply(us[i], g, B))
        assert metrics.rel_linf(got[i], ref) <= 2e-6
        assert metrics.rel_l2(got[i], ref) <= 5e-7


def test_fp32_complex_apply_bound(api):
    n = 64
    rng = np.random.default_rng(9)
    v = (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) * synth.cutoff(n)
    plan = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("helm20"))
    got = plan.apply(_gpu(v, torch.complex64)).cpu().numpy().astype(np.complex128)
    ref = scheme.apply(v, oracle_table("helm20", n), B)
    assert metrics.rel_linf(got, ref) <= 2e-6


def test_in_place_and_empty_batch_and_determinism(api):
    n = 128
    u = synth.smooth_density(n, 1010)
    plan = api.ConvPlan(n=n, **plan_kwargs("pow-1/2"))
    t = _gpu(u, torch.float64).unsqueeze(0).contiguous()
    a = plan.apply(t.clone()).cpu().numpy()
    b = plan.apply(t.clone()).cpu().numpy()
    assert np.array_equal(a, b)                            # bitwise reproducible
    tt = t.clone()
    plan.apply(tt, out=tt)                                 # in place
    assert np.array_equal(tt.cpu().numpy(), a)
    empty = torch.empty((0, n, n), dtype=torch.float64, device="cuda")
    assert plan.apply(empty).shape == (0, n, n)


def test_batch_independence(api):
    # Each density's result is the same alone and inside a batch (bitwise).
    n = 64
    us = np.stack([synth.smooth_density(n, 1020 + i) for i in range(5)])
    plan = api.ConvPlan(n=n, **plan_kwargs("log"))
    allb = plan.apply(_gpu(us, torch.float64)).cpu().numpy()
    for i in (0, 3):
        one = plan.apply(_gpu(us[i:i + 1], torch.float64)).cpu().numpy()[0]
        assert np.array_equal(one, allb[i])


@pytest.mark.parametrize("n", [16, 32])
def test_ls_solve_fp64_vs_dense(api, n):
    kappa = 20.0
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(3020))
    plan = api.ConvPlan(n=n, **plan_kwargs("helm20"))
    u, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-12, restart=20)
    assert info.status == 0, info
    g = oracle_table("helm20", n)
    ref = ols.dense_solve(m, ui, g, B, kappa)
    got = u.cpu().numpy()
    assert metrics.rel_linf(got, ref) <= 1e-10
    res = ui - ols.matvec(got, m, g, B, kappa)
    assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1e-11


@pytest.mark.parametrize("n", [32, 64])
def test_ls_solve_mixed_precision(api, n):
    kappa = 40.0
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(3040))
    plan = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("helm40"))
    u, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-8, restart=30,
                            mixed=True)
    assert info.status == 0, info
    assert info.refinements >= 1
    g = oracle_table("helm40", n)
    got = u.cpu().numpy()
    res = ui - ols.matvec(got, m, g, B, kappa)
    assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1.2e-8
    ref, oinfo = ols.gmres(m, ui, g, B, kappa, tol=1e-12, restart=50)
    assert metrics.rel_linf(got, ref) <= 1e-6


def test_ls_zero_contrast_and_zero_rhs(api):
    n, kappa = 32, 20.0
    plan = api.ConvPlan(n=n, **plan_kwargs("helm20"))
    ui = synth.plane_wave(n, kappa, 0.3)
    u, info = plan.ls_solve(_gpu(np.zeros((n, n)), torch.float64), _gpu(ui, torch.complex128), tol=1e-10)
    assert info.status == 0 and np.max(np.abs(u.cpu().numpy() - ui)) < 1e-14
    z, info = plan.ls_solve(_gpu(synth.contrast(n), torch.float64),
                            torch.zeros((n, n), dtype=torch.complex128, device="cuda"), tol=1e-10)
    assert info.status == 0 and info.matvecs == 0 and torch.all(z == 0)


def test_ls_maxit_status(api):
    n, kappa = 32, 40.0
    plan = api.ConvPlan(n=n, **plan_kwargs("helm40"))
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, 0.3)
    u, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-14, restart=5,
                            max_matvecs=7)
    assert info.status == 1 and info.matvecs <= 8 and info.rel_residual > 1e-14


# Densities of different sizes and kernels in shared launches (conv_apply_multi).
MULTI_REAL = [("log", 64, 3), ("pow-1/2", 128, 2), ("pow-1/3", 16, 5), ("log", 512, 1), ("log", 32, 4),
              ("pow-1/2", 256, 2), ("log", 16, 1), ("pow-1/3", 1024, 1), ("log", 2048, 3), ("pow-1/2", 64, 2)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_apply_multi_uneven_sizes_real(api, precision):
    dt = torch.float64 if precision == "fp64" else torch.float32
    plans = [api.ConvPlan(n=n, precision=precision, **plan_kwargs(k)) for k, n, _ in MULTI_REAL]
    hosts = [np.stack([synth.smooth_density(n, 1300 + 10 * i + j) for j in range(b)])
             for i, (_, n, b) in enumerate(MULTI_REAL)]
    dens = [_gpu(h, dt) for h in hosts]
    outs = api.apply_multi(plans, dens)            # 10 items: more than one launch per pass
    # The same arithmetic as a single-plan apply, compiled into a different kernel
    # (another block shape), so results agree to rounding rather than bitwise.
    same = 1e-14 if precision == "fp64" else 2e-6
    for (k, n, b), p, d, o in zip(MULTI_REAL, plans, dens, outs):
        one = p.apply(d).cpu().numpy().astype(np.float64)
        got = o.cpu().numpy().astype(np.float64)
        assert metrics.rel_linf(got, one) <= same, (k, n)
        # against the oracle where its moment table is cheap (the power-kernel table is
        # a quadrature per distinct |k|: minutes of CPU above n = 256)
        if n > (1024 if k == "log" else 256):
            continue
        for j in range(b):
            ref = np.real(scheme.apply(hosts[MULTI_REAL.index((k, n, b))][j], oracle_table(k, n), B))
            if precision == "fp64":
                assert metrics.rel_linf(got[j], ref) <= FP64_TOL, (k, n, j)
            else:
                assert metrics.rel_linf(got[j], ref) <= 2e-6 and metrics.rel_l2(got[j], ref) <= 5e-7, (k, n, j)


def test_apply_multi_uneven_sizes_complex(api):
    specs = [("helm20", 64, 2), ("helm40", 128, 1), ("helm20", 16, 3), ("helm40", 256, 2)]
    plans = [api.ConvPlan(n=n, **plan_kwargs(k)) for k, n, _ in specs]
    rng = np.random.default_rng(77)
    hosts = [(rng.normal(size=(b, n, n)) + 1j * rng.normal(size=(b, n, n))) * synth.cutoff(n) for _, n, b in specs]
    dens = [_gpu(h, torch.complex128) for h in hosts]
    outs = api.apply_multi(plans, dens)
    for (k, n, b), p, d, o, h in zip(specs, plans, dens, outs, hosts):
        assert metrics.rel_linf(o.cpu().numpy(), p.apply(d).cpu().numpy()) <= 1e-14, (k, n)
        for j in range(b):
            ref = scheme.apply(h[j], oracle_table(k, n), B)
            assert metrics.rel_linf(o[j].cpu().numpy(), ref) <= FP64_TOL, (k, n, j)


def test_apply_multi_rejects_mixed_kinds(api):
    from paper_2107_03958_amd import _lib as L
    a = api.ConvPlan(n=32, **plan_kwargs("log"))
    b = api.ConvPlan(n=32, **plan_kwargs("helm20"))
    c = api.ConvPlan(n=32, precision="fp32", **plan_kwargs("log"))
    u = torch.zeros((1, 32, 32), dtype=torch.float64, device="cuda")
    with pytest.raises(L.WsError):
        api.apply_multi([a, b], [u, u.to(torch.complex128)])
    with pytest.raises(L.WsError):
        api.apply_multi([a, c], [u, u.float()])


def test_ls_graph_replays_match_eager(api, monkeypatch):
    # GMRES steps replayed from captured graphs give the eager launches' results,
    # replay after replay, with other GPU work and synchronisations in between,
    # on the null stream and on a side stream.
    n, kappa = 64, 40.0
    m = _gpu(synth.contrast(n), torch.float64)
    ui = _gpu(synth.plane_wave(n, kappa, 0.9), torch.complex128)
    monkeypatch.setenv("WSCONV_LS_GRAPHS", "0")
    eager = api.ConvPlan(n=n, **plan_kwargs("helm40"))
    monkeypatch.delenv("WSCONV_LS_GRAPHS")
    graph = api.ConvPlan(n=n, **plan_kwargs("helm40"))
    for mixed, prec in ((False, "fp64"), (True, "fp32")):
        pe = eager if not mixed else None
        if mixed:
            monkeypatch.setenv("WSCONV_LS_GRAPHS", "0")
            pe = api.ConvPlan(n=n, precision="fp32", **plan_kwargs("helm40"))
            monkeypatch.delenv("WSCONV_LS_GRAPHS")
        pg = graph if not mixed else api.ConvPlan(n=n, precision="fp32", **plan_kwargs("helm40"))
        ref, iref = pe.ls_solve(m, ui, tol=1e-10, restart=20, mixed=mixed)
        work = pg.ls_workspace(20, mixed)
        out = torch.empty_like(ui)
        noise = api.ConvPlan(n=128, **plan_kwargs("log"))
        side = torch.cuda.Stream()
        for rep in range(4):
            got, info = pg.ls_solve(m, ui, tol=1e-10, restart=20, mixed=mixed, out=out, work=work)
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (prec, rep)
            assert info.matvecs == iref.matvecs and info.status == 0
            noise.apply(torch.randn((2, 128, 128), dtype=torch.float64, device="cuda"))   # eager work between
            torch.cuda.synchronize()
        with torch.cuda.stream(side):
            got, info = pg.ls_solve(m, ui, tol=1e-10, restart=20, mixed=mixed, work=work,
                                    stream=side)
        side.synchronize()
        assert torch.equal(got, ref), prec
