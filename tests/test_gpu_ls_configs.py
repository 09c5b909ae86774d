"""Lippmann-Schwinger solves at the benchmark's own sizes, and the solver's
breakdown status, through the C-ABI against the CPU oracle.

Workload (Section 3.3, eq. descretls): Helmholtz kernel, contrast
m = 0.5 cut(r), plane wave at the seeded angle of each kappa; GMRES(50).
The GPU solves to a true relative residual of 1e-12 in FP64, and in FP32
with FP64 iterative refinement; the oracle's own FP64 GMRES solves the same
discrete system to 1e-13.

Reading of the bar for an iterative solve.  Two approximate solutions of
K x = f with true relative residuals r1 and r2 differ by at most
cond_2(K) (r1 + r2) in the relative 2-norm (x1 - x2 = K^-1 (res2 - res1)).
cond_2(K) of the discrete operator is measured by the oracle's dense SVD
(tests/test_oracle_smoothing_ls.py checks the table COND_BOUND at n = 32;
it converges in n: 8.49 / 8.38 / 8.34 at kappa = 20 and n = 16 / 32 / 64).
So the checks are: the GPU solution's residual recomputed with the oracle's
operator meets the requested tolerance (to rounding), and the GPU and oracle
solutions agree within 2 COND_BOUND (r_gpu + r_oracle) in relative L-infinity
(the factor 2 covers L-infinity against the 2-norm on these smooth fields).
"""
import functools

import numpy as np
import pytest

import synth
from oracle import ls as ols
from oracle import metrics, moments
from tests.gpu_common import A_DEFAULT, B, COND_BOUND

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_2107_03958_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _api


def _gpu(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


@functools.lru_cache(maxsize=8)
def _oracle_case(n, kappa):
    g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A_DEFAULT)
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(synth.SEED_LS_ANGLE + int(kappa)))
    x, info = ols.gmres(m, ui, g, B, kappa, tol=1e-13, restart=50)
    assert info["converged"], info
    return m, ui, g, x, info["rel_residual"]


def _check_solve(api, n, kappa, mode):
    m, ui, g, xo, ro = _oracle_case(n, kappa)
    mixed = mode == "fp32+ir"
    print(f"ls case n={n} kappa={kappa} {mode}", flush=True)
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa, precision="fp32" if mixed else "fp64")
    u, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-12, restart=50,
                            mixed=mixed)
    assert info.status == 0, info
    if mixed:
        assert info.refinements >= 2, info
    got = u.cpu().numpy()
    res = np.linalg.norm(ui - ols.matvec(got, m, g, B, kappa)) / np.linalg.norm(ui)
    assert res <= 1.2e-12, (res, info)
    assert abs(res - info.rel_residual) <= 1e-14 + 0.05 * res, (res, info.rel_residual)
    bound = 2.0 * COND_BOUND[kappa] * (res + ro)
    err = metrics.rel_linf(got, xo)
    assert err <= bound, (err, bound, res, ro)


@pytest.mark.slow
@pytest.mark.parametrize("mode", ["fp64", "fp32+ir"])
@pytest.mark.parametrize("kappa", [20.0, 40.0, 80.0])
def test_ls_solve_n256(api, kappa, mode):
    _check_solve(api, 256, kappa, mode)


@pytest.mark.slow
@pytest.mark.parametrize("mode", ["fp64", "fp32+ir"])
def test_ls_solve_n512_kappa80(api, mode):
    _check_solve(api, 512, 80.0, mode)


@pytest.mark.slow
@pytest.mark.parametrize("mode", ["fp64", "fp32+ir"])
def test_ls_solve_n1024_kappa80_residual(api, mode):
    # the largest LS case of the benchmark: the GPU solution's residual recomputed with the
    # oracle's operator (one oracle matvec) meets the requested tolerance, so the solution is
    # within cond_2(K) times it of the discrete system's exact solution
    n, kappa = 1024, 80.0
    mixed = mode == "fp32+ir"
    print(f"ls case n={n} kappa={kappa} {mode}", flush=True)
    g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A_DEFAULT)
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(synth.SEED_LS_ANGLE + int(kappa)))
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa, precision="fp32" if mixed else "fp64")
    u, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-10, restart=50,
                            mixed=mixed)
    assert info.status == 0, info
    got = u.cpu().numpy()
    res = np.linalg.norm(ui - ols.matvec(got, m, g, B, kappa)) / np.linalg.norm(ui)
    assert res <= 1.2e-10, (res, info)
    assert abs(res - info.rel_residual) <= 1e-14 + 0.05 * res, (res, info.rel_residual)


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("kappa", [20.0, 40.0])
def test_ls_solve_fp64_vs_dense_tight(api, n, kappa):
    # Against the exact (LU) solution of the discrete system: with the GPU at a true
    # residual of 1e-14 and cond_2(K) <= COND_BOUND, the FP64 bar of 1e-12 holds.
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(synth.SEED_LS_ANGLE + int(kappa)))
    g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A_DEFAULT)
    ref = ols.dense_solve(m, ui, g, B, kappa)
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa)
    u, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-14, restart=50)
    assert info.status == 0, info
    assert COND_BOUND[kappa] * 2 * info.rel_residual <= 1e-12
    assert metrics.rel_linf(u.cpu().numpy(), ref) <= 1e-12


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("where", ["u_inc", "contrast"])
def test_ls_nonfinite_input_breaks_down(api, where, mixed):
    # A NaN in the data makes the residual non-finite: the solve stops with
    # WS_LS_BREAKDOWN (return value 2) instead of iterating to max_matvecs.
    n, kappa = 32, 20.0
    m = synth.contrast(n)
    ui = synth.plane_wave(n, kappa, 0.3)
    if where == "u_inc":
        ui[5, 7] = np.nan
    else:
        m[16, 16] = np.nan
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa, precision="fp32" if mixed else "fp64")
    _, info = plan.ls_solve(_gpu(m, torch.float64), _gpu(ui, torch.complex128), tol=1e-10, restart=20,
                            max_matvecs=400, mixed=mixed)
    assert info.status == 2, info
    assert info.matvecs <= 60, info
    # the plan is still usable afterwards
    m2 = synth.contrast(n)
    ui2 = synth.plane_wave(n, kappa, 0.3)
    _, info2 = plan.ls_solve(_gpu(m2, torch.float64), _gpu(ui2, torch.complex128), tol=1e-8, restart=20,
                             mixed=mixed)
    assert info2.status == 0, info2
