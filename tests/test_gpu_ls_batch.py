"""Several Lippmann-Schwinger solves of one plan run together (ls_solve_batch,
Section 3.3, eq. descretls) through the C-ABI.

Every GMRES instance of a batch keeps its own Hessenberg matrix, rotations,
stop test and budget, and the batched kernels compute each instance's
arithmetic exactly as the single-solve kernels do, so each batched solution
must equal its alone solution (ls_solve) bitwise, with the same counters.
The solutions also meet the requested tolerance on the oracle's operator.
"""
import numpy as np
import pytest

import synth
from oracle import ls as ols
from oracle import moments
from tests.gpu_common import A_DEFAULT, B

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_2107_03958_amd import api as _api
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _api


def _inputs(n, kappa, count, seed):
    rng = np.random.default_rng(seed)
    ms = np.stack([rng.uniform(0.2, 0.8) * synth.cutoff(n) for _ in range(count)])
    uis = np.stack([synth.plane_wave(n, kappa, rng.uniform(0, 2 * np.pi)) for _ in range(count)])
    return ms, uis


def _gpu(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("mixed", [False, True])
def test_batch_equals_alone(api, mixed):
    n, kappa, count = 64, 40.0, 5
    print(f"ls batch n={n} kappa={kappa} count={count} mixed={mixed}", flush=True)
    ms, uis = _inputs(n, kappa, count, 77)
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa, precision="fp32" if mixed else "fp64")
    tol = 1e-10
    ub, infos = plan.ls_solve_batch(_gpu(ms, torch.float64), _gpu(uis, torch.complex128), tol=tol, restart=20,
                                    mixed=mixed)
    got = ub.cpu().numpy()
    g = moments.ghat_table(moments.Kernel("helmholtz", 1.0, 0.0, kappa), n, B, A_DEFAULT)
    for s in range(count):
        ua, ia = plan.ls_solve(_gpu(ms[s], torch.float64), _gpu(uis[s], torch.complex128), tol=tol, restart=20,
                               mixed=mixed)
        assert infos[s].status == 0 and ia.status == 0, (infos[s], ia)
        assert (infos[s].matvecs, infos[s].iterations, infos[s].refinements) == (ia.matvecs, ia.iterations,
                                                                                 ia.refinements)
        assert np.array_equal(got[s], ua.cpu().numpy()), s
        res = np.linalg.norm(uis[s] - ols.matvec(got[s], ms[s], g, B, kappa)) / np.linalg.norm(uis[s])
        assert res <= 1.05 * tol, (s, res)


def test_batch_mixed_outcomes(api):
    # A zero right-hand side (done at once), a NaN (breakdown), a tight budget (max_matvecs) and
    # ordinary solves in one batch: the outcomes stay per solve, and the ordinary solves still
    # equal their alone results.
    n, kappa, count = 32, 20.0, 4
    print(f"ls batch outcomes n={n} count={count}", flush=True)
    ms, uis = _inputs(n, kappa, count, 78)
    uis[1] = 0.0
    uis[2, 3, 3] = np.nan
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa)
    ub, infos = plan.ls_solve_batch(_gpu(ms, torch.float64), _gpu(uis, torch.complex128), tol=1e-12, restart=10,
                                    max_matvecs=200)
    assert infos[1].status == 0 and infos[1].matvecs == 0
    assert infos[2].status == 2
    for s in (0, 3):
        ua, ia = plan.ls_solve(_gpu(ms[s], torch.float64), _gpu(uis[s], torch.complex128), tol=1e-12, restart=10,
                               max_matvecs=200)
        assert infos[s].status == ia.status == 0 and infos[s].matvecs == ia.matvecs
        assert np.array_equal(ub[s].cpu().numpy(), ua.cpu().numpy())
    assert torch.all(ub[1] == 0)
    # a budget that stops every solve early
    ub, infos = plan.ls_solve_batch(_gpu(ms, torch.float64), _gpu(np.nan_to_num(uis), torch.complex128), tol=1e-14,
                                    restart=5, max_matvecs=7)
    for s in (0, 2, 3):
        assert infos[s].status == 1 and infos[s].matvecs <= 8, infos[s]


@pytest.mark.slow
def test_batch_n256_bench_size(api):
    n, kappa, count = 256, 40.0, 8
    print(f"ls batch n={n} kappa={kappa} count={count}", flush=True)
    ms, uis = _inputs(n, kappa, count, 79)
    plan = api.ConvPlan("helmholtz", n=n, kappa=kappa)
    ub, infos = plan.ls_solve_batch(_gpu(ms, torch.float64), _gpu(uis, torch.complex128), tol=1e-8, restart=50)
    for s in (0, count - 1):
        ua, ia = plan.ls_solve(_gpu(ms[s], torch.float64), _gpu(uis[s], torch.complex128), tol=1e-8, restart=50)
        assert infos[s].status == 0 and infos[s].matvecs == ia.matvecs
        assert np.array_equal(ub[s].cpu().numpy(), ua.cpu().numpy())


def test_batch_rejects_bad_counts(api):
    from paper_2107_03958_amd import _lib as L
    plan = api.ConvPlan("helmholtz", n=16, kappa=20.0)
    import ctypes
    nb = ctypes.c_size_t()
    assert plan.lib.ls_solve_batch_query(plan.handle, 0, 20, 0, ctypes.byref(nb)) == L.WS_EINVAL
    assert plan.lib.ls_solve_batch_query(plan.handle, 65, 20, 0, ctypes.byref(nb)) == L.WS_EINVAL
    assert plan.lib.ls_solve_batch_query(plan.handle, 64, 20, 0, ctypes.byref(nb)) == L.WS_OK
