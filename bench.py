#!/usr/bin/env python3
"""Benchmark of the FFT apply of A_n and of the Lippmann-Schwinger solve on one MI355X.

Workload (one "step"): 32 seeded smooth densities (sums of 1..8 Gaussian bumps
times the C-infinity cutoff) on a 2048 x 2048 grid of D, periodic extension
b = 2 (4096 x 4096 FFT), applied with each of the kernels log|x|, |x|^-1/2 and
|x|^-1/3: 96 applies per step, inputs resident in HBM, moments precomputed
in the plans.  The headline value is FP64 applies/s; the same step in FP32
(hi/lo twiddles) and the LS solve latencies (GMRES(50), tol 1e-8, FP64 and
FP32 + FP64 refinement) are reported beside it, with the roofline of the
dominant kernel (timed live with HIP events) and the CPU oracle timed on a
bounded sample on the host.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "conv applies/s + HBM GB/s at 2048² FP64 vs FP32; p50/p99 LS solve latency"
PEAK_HBM_GBPS = 8000.0
KERNELS = [
    ("log|x|", dict(family="log", scale=1.0)),
    ("|x|^-1/2", dict(family="power", scale=1.0, gamma=-0.5)),
    ("|x|^-1/3", dict(family="power", scale=1.0, gamma=-1.0 / 3.0)),
]
PASS_NAMES = ["k_rows_fwd_real", "k_cols", "k_rows_inv_real"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pass_bytes(n: int, s: int) -> list[float]:
    """Algorithmic HBM bytes of the three passes for one real density (s = bytes per real).

    pass 0 reads the n x n samples and writes the n x n complex half spectrum;
    pass 1 reads and writes that intermediate and reads the n(n+1) moments plus
    the n+1 of the packed Nyquist column; pass 2 reads the intermediate and writes
    n x n samples.  Their sum is the 11 n^2 s pass model of the apply.
    """
    return [3.0 * n * n * s, 4.0 * n * n * s + (n + 1) * (n + 1) * s, 3.0 * n * n * s]


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "apply_fp64_2048_traffic.json")


def measured_traffic(kernel: str, precision: str, n: int, chunk: int):
    """HBM bytes per launch of `kernel` from the committed PMC summary (FETCH_SIZE + WRITE_SIZE,
    calibrated by a copy of known size), or None when the summary does not describe these
    kernel sources, this precision or this launch shape."""
    from paper_2107_03958_amd import traffic
    if precision != "fp64" or n != 2048:
        return None
    res = traffic.load_for_current_sources(TRAFFIC_SUMMARY)
    if res is None or res.get("densities_per_dispatch") != chunk:
        return None
    for name, v in res["kernels"].items():
        if name.startswith("ws::" + kernel + "<double"):
            return v["traffic_bytes"]
    return None


def run_apply_bench(api, torch, n, batch, precision, steps, warmup, u_host):
    dt = torch.float64 if precision == "fp64" else torch.float32
    s = 8 if precision == "fp64" else 4
    stream = torch.cuda.current_stream()
    t_plan = []
    plans = []
    for name, kw in KERNELS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plans.append(api.ConvPlan(n=n, precision=precision, **kw))
        torch.cuda.synchronize()
        t_plan.append(time.perf_counter() - t0)
    u = u_host.to(dt).cuda()
    out = torch.empty_like(u)
    work = torch.empty(max(1, plans[0].chunk) * plans[0].work_bytes, dtype=torch.uint8, device="cuda")
    nk = len(plans)
    chunk = plans[0].chunk            # densities taken through all three passes at a time (as conv_apply)
    groups = [(b0, min(batch, b0 + chunk)) for b0 in range(0, batch, chunk)]
    ng = len(groups)
    # One event before and after each pass of each density group of each kernel, on the launch stream.
    ev = [[[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(nk * ng)] for _ in range(steps)]
    pass_ms = np.zeros(3)
    views = [(u[a:b], out[a:b]) for a, b in groups]

    def step(evs):
        for ki, p in enumerate(plans):
            for gi, (uv, ov) in enumerate(views):
                e = None if evs is None else evs[ki * ng + gi]
                if e is not None:
                    e[0].record(stream)
                for ps in range(3):
                    p.apply_pass(ps, uv, ov, work, stream)
                    if e is not None:
                        e[ps + 1].record(stream)

    for _ in range(warmup):
        step(None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(steps):
        step(ev[st])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for st in range(steps):
        for e in ev[st]:
            for ps in range(3):
                pass_ms[ps] += e[ps].elapsed_time(e[ps + 1])
    launches = steps * nk * ng
    avg_pass_ms = pass_ms / launches       # per launch of `chunk` densities
    applies = steps * nk * batch
    pb = pass_bytes(n, s)
    res = dict(
        applies_per_s=applies / elapsed,
        ms_per_step=elapsed / steps * 1e3,
        pass_model_gbps=applies * sum(pb) / elapsed / 1e9,
        pass_avg_ms={PASS_NAMES[i]: float(avg_pass_ms[i]) for i in range(3)},
        pass_gbps={PASS_NAMES[i]: float(pb[i] * batch * steps * nk / (pass_ms[i] * 1e-3) / 1e9) for i in range(3)},
        densities_per_launch=chunk,
        plan_build_s={KERNELS[i][0]: t_plan[i] for i in range(nk)},
    )
    dom = int(np.argmax(avg_pass_ms))
    per_launch = pb[dom] * batch / ng                  # algorithmic bytes of one launch (average group)
    achieved = per_launch / (avg_pass_ms[dom] * 1e-3) / 1e9
    res["roofline"] = dict(bound="hbm", kernel=PASS_NAMES[dom], achieved=achieved, peak=PEAK_HBM_GBPS,
                           unit="GB/s", frac=achieved / PEAK_HBM_GBPS,
                           traffic=measured_traffic(PASS_NAMES[dom], precision, n, chunk),
                           bytes_per_launch=per_launch, launch_avg_ms=float(avg_pass_ms[dom]))
    # Keep the last outputs of the first kernel for the FP32-vs-FP64 comparison.
    plans[0].apply(u, out=out, work=work)
    res["_out_first_kernel"] = out[:4].double().cpu().numpy()
    return res


def run_ls_bench(api, torch, ns, kappas, repeats):
    import synth
    lat = {"fp64": [], "fp32+ir": []}
    detail = []
    for n in ns:
        for kappa in kappas:
            m = torch.as_tensor(synth.contrast(n)).cuda()
            theta = synth.plane_wave_angle(synth.SEED_LS_ANGLE + int(kappa))
            ui = torch.as_tensor(synth.plane_wave(n, kappa, theta)).cuda()
            for mode in ("fp64", "fp32+ir"):
                mixed = mode != "fp64"
                plan = api.ConvPlan("helmholtz", n=n, kappa=kappa, precision="fp32" if mixed else "fp64")
                work = plan.ls_workspace(50, mixed)
                out = torch.empty_like(ui)
                plan.ls_solve(m, ui, tol=1e-8, restart=50, mixed=mixed, out=out, work=work)  # warm-up
                for _ in range(repeats):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, info = plan.ls_solve(m, ui, tol=1e-8, restart=50, mixed=mixed, out=out, work=work)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    lat[mode].append(dt)
                detail.append(dict(n=n, kappa=kappa, mode=mode, ms=dt * 1e3, matvecs=info.matvecs,
                                   iterations=info.iterations, refinements=info.refinements,
                                   rel_residual=info.rel_residual, status=info.status))
                log(f"ls n={n} kappa={kappa} {mode}: {dt * 1e3:.2f} ms, matvecs={info.matvecs}, "
                    f"rel_res={info.rel_residual:.2e}, status={info.status}")
    out = {}
    for mode, v in lat.items():
        v = np.array(v) * 1e3
        out[mode] = dict(p50_ms=float(np.percentile(v, 50)), p99_ms=float(np.percentile(v, 99)), solves=len(v))
    out["cases"] = detail
    return out


def cpu_baseline(n, u0):
    """The oracle (plain FP64 CPU) on one density of the workload: moments + apply, one thread."""
    from threadpoolctl import threadpool_limits

    from oracle import moments, scheme
    a = (2 + math.sqrt(2) / 2 - 0.5) / 2
    with threadpool_limits(1):
        t0 = time.perf_counter()
        g = moments.ghat_table(moments.Kernel("log", 1.0), n, 2, a)
        t1 = time.perf_counter()
        r = np.real(scheme.apply(u0, g, 2))
        t2 = time.perf_counter()
    # The GPU value excludes the one-time moment precompute (plans are built before timing), so
    # the baseline rate is the oracle's apply alone; its moment-table time is reported beside it.
    return dict(value=1.0 / (t2 - t1), unit="applies/s", cores=1, kind="oracle",
                sample=f"1 density of the {n}x{n} workload, kernel log|x|: apply with the oracle's own "
                       f"radix-4/2 FFT ({t2 - t1:.1f} s, one thread); its moment table took {t1 - t0:.1f} s",
                moment_s=t1 - t0, apply_s=t2 - t1), r


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ls", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--ls-n", type=int, nargs="*", default=[256, 512])
    ap.add_argument("--ls-kappa", type=float, nargs="*", default=[20.0, 40.0, 80.0])
    ap.add_argument("--ls-repeats", type=int, default=3)
    args = ap.parse_args(argv)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; every workload is per-density "
                                   "independent and would shard by density across GPUs (see DESIGN.md)",
                          "n_gpus": args.gpus}))
        return 2

    import torch

    import synth
    from paper_2107_03958_amd import _lib, api
    _lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, batch = args.n, args.batch

    log(f"generating {batch} densities at n={n} ...")
    u_host = torch.as_tensor(np.stack([synth.smooth_density(n, synth.SEED_PRECISION + i) for i in range(batch)]))

    log("FP64 apply bench ...")
    r64 = run_apply_bench(api, torch, n, batch, "fp64", args.steps, args.warmup, u_host)
    log(f"fp64: {r64['applies_per_s']:.1f} applies/s, pass model {r64['pass_model_gbps']:.0f} GB/s, "
        f"passes {r64['pass_avg_ms']}")
    out64 = r64.pop("_out_first_kernel")
    r32 = None
    if not args.no_fp32:
        log("FP32 apply bench ...")
        r32 = run_apply_bench(api, torch, n, batch, "fp32", args.steps, args.warmup, u_host)
        out32 = r32.pop("_out_first_kernel")
        diff = out32 - out64
        r32["rel_linf_vs_fp64_gpu"] = float(np.max(np.abs(diff)) / np.max(np.abs(out64)))
        r32["rel_l2_vs_fp64_gpu"] = float(np.linalg.norm(diff) / np.linalg.norm(out64))
        log(f"fp32: {r32['applies_per_s']:.1f} applies/s, pass model {r32['pass_model_gbps']:.0f} GB/s")
    ls = None
    if not args.no_ls:
        log("LS latency bench ...")
        ls = run_ls_bench(api, torch, args.ls_n, args.ls_kappa, args.ls_repeats)
    cpu = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (bounded sample) ...")
        cpu, ref = cpu_baseline(n, u_host[0].numpy())
        cpu["gpu_fp64_rel_linf_vs_oracle"] = float(np.max(np.abs(out64[0] - ref)) / np.max(np.abs(ref)))
        log(f"cpu oracle: {cpu['value']:.4f} applies/s; GPU FP64 vs oracle rel Linf "
            f"{cpu['gpu_fp64_rel_linf_vs_oracle']:.2e}")

    line = {
        "metric": METRIC,
        "value": r64["applies_per_s"],
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"A_n apply, {n}x{n} grid on D, period b=2 ({2 * n}^2 FFT), {batch} smooth "
                        f"densities x {len(KERNELS)} kernels per step, FP64, inputs resident in HBM",
            "grid": n, "fft": 2 * n, "batch_per_kernel": batch, "kernels": [k for k, _ in KERNELS],
        },
        "grid_points_per_s": r64["applies_per_s"] * n * n,
        "hbm_gbps_pass_model": r64["pass_model_gbps"],
        "hbm_frac_pass_model": r64["pass_model_gbps"] / PEAK_HBM_GBPS,
        "pass_avg_ms": r64["pass_avg_ms"],
        "pass_gbps": r64["pass_gbps"],
        "plan_build_s": r64["plan_build_s"],
        "roofline": r64["roofline"],
    }
    if r32 is not None:
        line["fp32"] = {k: r32[k] for k in ("applies_per_s", "ms_per_step", "pass_model_gbps", "pass_avg_ms",
                                            "pass_gbps", "rel_linf_vs_fp64_gpu", "rel_l2_vs_fp64_gpu",
                                            "roofline")}
    if ls is not None:
        line["ls_latency"] = ls
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
