"""Serving engine on the GPU (include/wsserve.h), through the C-ABI.

- A mix of applies and LS solves of different sizes and kernels, submitted at
  once to an engine with several streams and batching, gives for every request
  the result the same request gets when served alone (one stream, no batching).
- The FP32 engine's results meet the FP32 apply bounds against the oracle and
  the LS residual target, the FP64 engine's meet the FP64 bar.
- Admission by footprint with an arena that holds one large job at a time,
  plan eviction, and rejection of a request larger than the arena.
"""
import numpy as np
import pytest

import synth
from oracle import ls as ols
from oracle import metrics, scheme
from tests.gpu_common import B, oracle_table, plan_kwargs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def serve():
    from paper_2107_03958_amd import serve as _serve
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return _serve


def _pinned(a, dtype):
    t = torch.empty(a.shape, dtype=dtype, pin_memory=True)
    t.copy_(torch.as_tensor(np.ascontiguousarray(a)))
    return t


def _mix_requests():
    """(kind, kernel name, n, inputs...) of a mixed workload; applies repeat per plan so they batch."""
    reqs = []
    for n in (64, 128, 256):
        for kname in ("log", "pow-1/2", "helm20"):
            for i in range(3):
                u = synth.smooth_density(n, 1000 + 10 * n + i)
                if kname == "helm20":
                    u = u * (1.0 + 0.5j)
                reqs.append(("apply", kname, n, u))
    for n, kname, kappa in ((32, "helm20", 20.0), (64, "helm40", 40.0), (32, "helm40", 40.0)):
        m = synth.contrast(n)
        ui = synth.plane_wave(n, kappa, synth.plane_wave_angle(3000 + int(kappa)))
        reqs.append(("ls", kname, n, m, ui, kappa))
    return reqs


def _request(eng, r):
    """The engine request of r, its page-locked inputs and output allocated."""
    if r[0] == "apply":
        kind, kname, n, u = r
        dt = torch.complex128 if np.iscomplexobj(u) else torch.float64
        return eng.request_apply(plan_kwargs(kname), _pinned(u, dt))
    kind, kname, n, m, ui, kappa = r
    return eng.request_ls(kappa, _pinned(m, torch.float64), _pinned(ui, torch.complex128), tol=1e-10, restart=30)


def _submit(eng, r):
    return eng.submit_request(*_request(eng, r))


def _run(eng, reqs, together):
    outs = []
    if together:
        # every request prepared first (page-locked buffers take time to allocate),
        # then submitted back to back, so the engine finds them pending together
        prepared = [_request(eng, r) for r in reqs]
        tickets = [eng.submit_request(req, held) for req, held in prepared]
        outs = [eng.wait(t, timeout=120) for t in tickets]
    else:
        for r in reqs:
            outs.append(eng.wait(_submit(eng, r), timeout=120))
    assert all(o is not None for o in outs), "a request timed out"
    return [(o[0].numpy().copy(), o[1]) for o in outs]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mix_equals_alone(serve, precision):
    reqs = _mix_requests()
    mix = serve.Engine(precision, streams=3, max_batch=4, arena_bytes=2 << 30)
    got = _run(mix, reqs, together=True)
    st = mix.stats()
    mix.close()
    alone_eng = serve.Engine(precision, streams=1, max_batch=1, arena_bytes=2 << 30)
    alone = _run(alone_eng, reqs, together=False)
    alone_eng.close()
    assert st["completed"] == len(reqs) and st["launches"] < len(reqs)    # some launches were batched
    assert max(info["batch"] for _, info in got) > 1
    assert all(info["batch"] == 1 for _, info in alone)
    for (a, ia), (b, ib), r in zip(got, alone, reqs):
        assert ia["status"] == 0 and ib["status"] == 0, r[:3]
        # same kernels, same arithmetic per density: identical results
        assert np.array_equal(a, b), r[:3]


def test_fp64_engine_vs_oracle(serve):
    eng = serve.Engine("fp64", streams=2, max_batch=4, arena_bytes=1 << 30)
    reqs = [r for r in _mix_requests() if r[0] == "ls" or r[2] <= 128]
    got = _run(eng, reqs, together=True)
    eng.close()
    for (out, info), r in zip(got, reqs):
        if r[0] == "apply":
            ref = scheme.apply(r[3], oracle_table(r[1], r[2]), B)
            ref = ref if np.iscomplexobj(r[3]) else np.real(ref)
            assert metrics.rel_linf(out, ref) <= 1e-12, r[:3]
        else:
            _, kname, n, m, ui, kappa = r
            g = oracle_table(kname, n)
            res = ui - ols.matvec(out, m, g, B, kappa)
            assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1.2e-10
            assert info["rel_residual"] <= 1e-10


def test_fp32_engine_vs_oracle(serve):
    eng = serve.Engine("fp32", streams=2, max_batch=4, arena_bytes=1 << 30)
    reqs = [r for r in _mix_requests() if r[0] == "ls" or r[2] <= 128]
    got = _run(eng, reqs, together=True)
    eng.close()
    for (out, info), r in zip(got, reqs):
        if r[0] == "apply":
            ref = scheme.apply(r[3], oracle_table(r[1], r[2]), B)
            ref = ref if np.iscomplexobj(r[3]) else np.real(ref)
            assert metrics.rel_linf(out, ref) <= 2e-6, r[:3]
            assert metrics.rel_l2(out, ref) <= 5e-7, r[:3]
        else:
            _, kname, n, m, ui, kappa = r
            g = oracle_table(kname, n)
            res = ui - ols.matvec(out, m, g, B, kappa)
            # FP32 inner solves, FP64 refinement: the true residual meets the target
            assert np.linalg.norm(res) / np.linalg.norm(ui) <= 1.2e-10
            assert info["refinements"] >= 1


def test_admission_tight_arena_and_eviction(serve):
    from paper_2107_03958_amd import _lib as L
    n, kappa = 128, 20.0
    m = _pinned(synth.contrast(n), torch.float64)
    ui = _pinned(synth.plane_wave(n, kappa, 0.7), torch.complex128)
    probe = serve.Engine("fp64", streams=1, max_batch=1, arena_bytes=1 << 20)
    req, _ = probe.request_ls(kappa, m, ui, tol=1e-10, restart=30)
    one_ls = probe.footprint(req)
    big = torch.zeros((512, 512), dtype=torch.float64)
    with pytest.raises(L.WsError):
        probe.submit_apply(plan_kwargs("log"), big)          # footprint above the 1 MiB arena
    probe.close()
    # room for one LS job plus 2 MiB (small applies fit beside it, a second LS job does not);
    # two plans at most
    slack = 2 << 20
    assert one_ls > 2 * slack
    eng = serve.Engine("fp64", streams=3, max_batch=2, max_plans=2, arena_bytes=one_ls + slack)
    tickets = [eng.submit_ls(kappa, m, ui, tol=1e-10, restart=30) for _ in range(3)]
    us = [synth.smooth_density(32, 1200 + i) for i in range(4)]
    kn = ["log", "pow-1/2", "pow-1/3", "log"]
    tickets += [eng.submit_apply(plan_kwargs(k), _pinned(u, torch.float64)) for k, u in zip(kn, us)]
    outs = [eng.wait(t, timeout=120) for t in tickets]
    st = eng.stats()
    eng.close()
    assert all(o is not None and o[1]["status"] == 0 for o in outs)
    assert st["arena_peak_bytes"] <= st["arena_bytes"]
    assert st["plan_evictions"] >= 1 and st["cached_plans"] <= 2
    ls_runs = sorted((o[1]["t_start"], o[1]["t_done"]) for o in outs[:3])
    for (s0, d0), (s1, d1) in zip(ls_runs, ls_runs[1:]):
        assert s1 >= d0 - 1e-3          # the three LS jobs did not overlap: one fits at a time
    a = outs[0][0].numpy()
    for o in outs[1:3]:
        assert np.array_equal(o[0].numpy(), a)
    for (out, _), k, u in zip(outs[3:], kn, us):
        ref = np.real(scheme.apply(u, oracle_table(k, 32), B))
        assert metrics.rel_linf(out.numpy(), ref) <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_mixed_plan_launches(serve, precision):
    # With mix_plans, applies of different sizes and kernels share launches
    # (conv_apply_multi).  Each result equals the request served alone to
    # rounding: the same arithmetic, compiled into another kernel.
    reqs = [r for r in _mix_requests() if r[0] == "apply"]
    eng = serve.Engine(precision, streams=2, max_batch=8, arena_bytes=2 << 30, mix_plans=True)
    # build every plan first, so the mixed batches below can form
    _run(eng, [reqs[i] for i in range(0, len(reqs), 3)], together=False)
    got = _run(eng, reqs, together=True)
    eng.close()
    alone_eng = serve.Engine(precision, streams=1, max_batch=1, arena_bytes=2 << 30)
    alone = _run(alone_eng, reqs, together=False)
    alone_eng.close()
    tol = 1e-13 if precision == "fp64" else 2e-6
    for (a, ia), (b, _), r in zip(got, alone, reqs):
        assert ia["status"] == 0
        assert metrics.rel_linf(a, b) <= tol, r[:3]
    # launches joined several requests (how many depends on how fast the
    # workers drain the queue, so only "more than one" is certain)
    assert max(info["batch"] for _, info in got) > 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ls_requests_batch(serve, precision):
    # LS solves with one plan and one setting that wait together run as one batched
    # solve (ls_solve_batch); each result equals the same request served alone.
    n, kappa, count = 64, 20.0, 7
    rng = np.random.default_rng(5)
    reqs = [("ls", "helm20", n, rng.uniform(0.2, 0.8) * synth.cutoff(n),
             synth.plane_wave(n, kappa, rng.uniform(0, 2 * np.pi)), kappa) for _ in range(count)]
    print(f"serve LS batch {precision} n={n} count={count}", flush=True)
    eng = serve.Engine(precision, streams=1, max_batch=8, arena_bytes=1 << 30)
    got = _run(eng, reqs, together=True)
    st = eng.stats()
    eng.close()
    alone_eng = serve.Engine(precision, streams=1, max_batch=1, arena_bytes=1 << 30)
    alone = _run(alone_eng, reqs, together=False)
    alone_eng.close()
    assert max(info["batch"] for _, info in got) > 1 and st["launches"] < count
    for (a, ia), (b, ib) in zip(got, alone):
        assert ia["status"] == 0 and ib["status"] == 0
        assert np.array_equal(a, b)
