"""Autotuner for the apply kernels' compile-time tile shapes.

The tile shapes (column-block width CB, rows per row tile RPB, elements per
thread ER/EC (and ERF, the forward real row pass's own ER), which fix the radix
plan of every line, the column-tile mapping
CPB, the smallest block WS_MIN_BLOCK and the chunk of the intermediate kept in
the last-level cache) are template constants: they size register arrays and
LDS.  Tuning is therefore offline: variant libraries are compiled with -D
overrides, each is timed on the GPU in a process of its own, and the fastest
shapes are written to csrc/tuned.hpp, which the next build picks up.

    python -m paper_2107_03958_amd.autotune build --dir DIR [--jobs 8]      # CPU: compile the variants
    python -m paper_2107_03958_amd.autotune time  --dir DIR [--n 2048]      # GPU: time them -> DIR/results.json
    python -m paper_2107_03958_amd.autotune choose --dir DIR [--write]      # pick, write csrc/tuned.hpp

The variants are the current shapes and their coordinate neighbours (one
parameter changed at a time).  A variant whose result differs from the
baseline's beyond rounding (1e-13 FP64, 5e-6 FP32 relative) is rejected.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "csrc", "tuned.hpp")

# Parameters per precision and the values tried around the current one.
PARAMS = {
    "fp64": {"WS_CB64": [2, 4], "WS_RPB64": [1, 2, 4], "WS_ER64": [8, 16], "WS_ERF64": [8, 16], "WS_EC64": [8, 16],
             "WS_CPB64": [0, 1]},
    "fp32": {"WS_CB32": [2, 4, 8], "WS_RPB32": [1, 2, 4], "WS_ER32": [8, 16], "WS_ERF32": [8, 16], "WS_EC32": [8, 16],
             "WS_CPB32": [0, 1]},
    "both": {"WS_MIN_BLOCK": [64, 128, 256], "WS_CHUNK_BYTES": ["(64u<<20)", "(128u<<20)", "(192u<<20)"]},
}


def current() -> dict:
    """The shapes the sources build with now (tuned.hpp, else the defaults in the headers)."""
    vals = {}
    for f in ("plan.hpp", "apply_cfg.hpp", "tuned.hpp"):
        path = os.path.join(HERE, "csrc", f)
        if not os.path.exists(path):
            continue
        for m in re.finditer(r"^#define (WS_[A-Z0-9_]+) (.+)$", open(path).read(), flags=re.M):
            name, val = m.group(1), m.group(2).strip()
            if f == "tuned.hpp" or name not in vals:
                vals[name] = val.replace(" ", "")
    return vals


def variants() -> list[dict]:
    base = current()
    out = [dict(name="base", precision="both", defines={})]
    for prec, params in PARAMS.items():
        for p, values in params.items():
            for v in values:
                if str(v).replace(" ", "") == str(base.get(p)):
                    continue
                out.append(dict(name=f"{p}={v}".replace("(", "").replace(")", "").replace("<<", "sh"),
                                precision=prec, defines={p: v}))
    return out


def cmd_build(args):
    from . import build
    os.makedirs(args.dir, exist_ok=True)
    vs = variants()

    def one(v):
        lib = os.path.join(args.dir, f"lib_{v['name']}.so")
        try:
            build.build(jobs=1, out=lib, defines=[f"{k}={x}" for k, x in v["defines"].items()],
                        build_dir=os.path.join(args.dir, "b_" + v["name"]))
            return dict(v, lib=lib, built=True)
        except Exception as e:   # a shape that does not fit (e.g. LDS) is skipped
            return dict(v, lib=lib, built=False, error=str(e))

    with cf.ThreadPoolExecutor(max_workers=args.jobs) as ex:
        res = list(ex.map(one, vs))
    json.dump(dict(base=current(), variants=res), open(os.path.join(args.dir, "variants.json"), "w"), indent=1)
    for r in res:
        print(f"{r['name']:28s} {'ok' if r['built'] else 'FAILED'}", flush=True)


def time_one(lib: str, n: int, precision: str, reps: int, b: int = 2) -> dict:
    """Runs in a fresh process: load `lib`, time the three passes of one chunk (HIP events) of the
    log|x| plan at size n and period b."""
    import ctypes

    import numpy as np
    import torch

    from . import _lib
    probe = ctypes.CDLL(lib)
    for name in list(_lib.EXPORTS):
        if not hasattr(probe, name):
            del _lib.EXPORTS[name]
    _lib.load(lib)
    from . import api
    plan = api.ConvPlan("log", n=n, b=b, precision=precision)
    b = plan.chunk
    g = torch.Generator().manual_seed(0)
    u = torch.randn((b, n, n), dtype=torch.float64, generator=g).to(plan.dtype).cuda()
    out = torch.empty_like(u)
    work = plan.workspace(b)
    st = torch.cuda.current_stream()
    for _ in range(3):
        for ps in range(3):
            plan.apply_pass(ps, u, out, work, st)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
    for r in range(reps):
        ev[r][0].record(st)
        for ps in range(3):
            plan.apply_pass(ps, u, out, work, st)
            ev[r][ps + 1].record(st)
    torch.cuda.synchronize()
    t = np.zeros(3)
    for r in range(reps):
        for ps in range(3):
            t[ps] += ev[r][ps].elapsed_time(ev[r][ps + 1])
    per = t * 1e3 / (reps * b)
    o = out[0].double().cpu().numpy()
    return dict(us_per_density=[float(x) for x in per], total_us=float(per.sum()),
                sample=o[:: max(1, n // 16), :: max(1, n // 16)].ravel().tolist(), scale=float(np.abs(o).max()))


def cmd_time(args):
    meta = json.load(open(os.path.join(args.dir, "variants.json")))
    results = []
    for v in meta["variants"]:
        if not v["built"]:
            continue
        for prec in (["fp64", "fp32"] if v["precision"] == "both" else [v["precision"]]):
            cmd = [sys.executable, "-m", "paper_2107_03958_amd.autotune", "_time", v["lib"], str(args.n), prec,
                   str(args.reps)]
            p = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=os.path.dirname(HERE))
            if p.returncode != 0:
                print(f"{v['name']} {prec}: failed\n{p.stderr[-2000:]}", flush=True)
                continue
            r = json.loads(p.stdout.strip().splitlines()[-1])
            results.append(dict(name=v["name"], precision=prec, defines=v["defines"], **r))
            print(f"{v['name']:28s} {prec}: {r['total_us']:8.2f} us/density  passes "
                  f"{[round(x, 2) for x in r['us_per_density']]}", flush=True)
    json.dump(dict(n=args.n, results=results), open(os.path.join(args.dir, f"results_{args.n}.json"), "w"),
              indent=1)


def cmd_choose(args):
    import numpy as np
    meta = json.load(open(os.path.join(args.dir, "variants.json")))
    res = json.load(open(os.path.join(args.dir, f"results_{args.n}.json")))["results"]
    chosen = {}
    lines = []
    ok = {}
    base = {}
    for prec in ("fp64", "fp32"):
        rs = [r for r in res if r["precision"] == prec]
        base[prec] = next(r for r in rs if r["name"] == "base")
        tol = 1e-13 if prec == "fp64" else 5e-6
        ok[prec] = {}
        for r in rs:
            d = np.max(np.abs(np.array(r["sample"]) - np.array(base[prec]["sample"]))) / base[prec]["scale"]
            if d <= tol:
                ok[prec][r["name"]] = r
            else:
                print(f"rejected {r['name']} {prec}: differs from the baseline by {d:.2e}")
    # score of a variant: its time relative to the baseline, summed over the
    # precisions its parameter affects; per parameter keep the best value if it
    # gains more than 1%
    for v in meta["variants"]:
        if not v["defines"]:
            continue
        (k, val), = v["defines"].items()
        precs = ["fp64", "fp32"] if v["precision"] == "both" else [v["precision"]]
        if not all(v["name"] in ok[p] for p in precs):
            continue
        score = sum(ok[p][v["name"]]["total_us"] / base[p]["total_us"] for p in precs) / len(precs)
        if score < 0.99 and (k not in chosen or score < chosen[k][1]):
            chosen[k] = (val, score)
    for k, (val, score) in sorted(chosen.items()):
        lines.append(f"{k}: {val} ({100 * (1 - score):.1f}% faster at n = {args.n})")
    chosen = {k: v for k, (v, _) in chosen.items()}
    print("\n".join(lines) if lines else "the current shapes stay")
    if args.write:
        cur = meta["base"]
        keys = sorted(set(k for p in PARAMS.values() for k in p))
        out = args.out or TUNED
        with open(out, "w") as fh:
            fh.write("// Tile shapes chosen by paper_2107_03958_amd/autotune.py on MI355X (gfx950),\n"
                     f"// timing the three apply passes at n = {args.n}; one parameter changed at a time\n"
                     "// from the previous shapes, kept when more than 1% faster.\n#pragma once\n")
            for k in keys:
                v = chosen.get(k, cur.get(k))
                if v is None:
                    continue
                fh.write(f"#ifndef {k}\n#define {k} {v}\n#endif\n")
        print(f"wrote {out}")


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "_time":
        lib, n, prec, reps = argv[1], int(argv[2]), argv[3], int(argv[4])
        period = int(argv[5]) if len(argv) > 5 else 2
        print(json.dumps(time_one(lib, n, prec, reps, period)), flush=True)
        return 0
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--dir", required=True)
    b.add_argument("--jobs", type=int, default=8)
    t = sub.add_parser("time")
    t.add_argument("--dir", required=True)
    t.add_argument("--n", type=int, default=2048)
    t.add_argument("--reps", type=int, default=20)
    c = sub.add_parser("choose")
    c.add_argument("--dir", required=True)
    c.add_argument("--n", type=int, default=2048)
    c.add_argument("--write", action="store_true")
    c.add_argument("--out", default=None, help="header to write (default csrc/tuned.hpp)")
    args = ap.parse_args(argv)
    {"build": cmd_build, "time": cmd_time, "choose": cmd_choose}[args.cmd](args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
