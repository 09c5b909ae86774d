"""Measured HBM traffic of the apply kernels from rocprofv3 PMC counters.

Two modes:

* ``python paper_2107_03958_amd/traffic.py target [--precision fp64|fp32]
  [--n N] [--b B]``: a short workload to run under ``rocprofv3 --pmc
  FETCH_SIZE`` (then ``--pmc WRITE_SIZE``).  It applies the plan for log|x|
  (default FP64, n = 2048, b = 2) to two whole chunks of densities and then
  copies a 512 MiB device buffer, whose counters calibrate the byte scale.
* ``python paper_2107_03958_amd/traffic.py summarise FETCH_DIR WRITE_DIR OUT``:
  reads the two ``*_counter_collection.csv`` files, scales each kernel's
  average counter per dispatch by the copy's (known bytes / counter), and
  writes OUT.json (plus OUT.md) with a hash of the kernel sources, so a reader
  can tell whether the figures still describe the current kernels.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 512 * 1024 * 1024


# The translation units of the measured kernels and what they include.
KERNEL_SOURCES = ("csrc/apply_f64.hip", "csrc/apply_f32.hip", "csrc/apply_impl.hpp", "csrc/apply_cfg.hpp", "csrc/fft_core.hpp", "csrc/plan.hpp", "csrc/tuned.hpp",
                  "../include/wsconv.h")


def source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        f = os.path.normpath(os.path.join(HERE, rel))
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def target(precision: str = "fp64", n: int = 2048, b: int = 2) -> None:
    import numpy as np
    import torch

    if __package__:
        from . import api
    else:
        sys.path.insert(0, os.path.dirname(HERE))
        from paper_2107_03958_amd import api
    plan = api.ConvPlan("log", n=n, b=b, precision=precision)
    dt = torch.float64 if precision == "fp64" else torch.float32
    u = torch.as_tensor(np.random.default_rng(0).normal(size=(2 * plan.chunk, n, n))).to(dt).cuda()  # two whole chunks
    out = torch.empty_like(u)
    work = torch.empty(plan.chunk * plan.work_bytes, dtype=torch.uint8, device="cuda")
    plan.apply(u, out=out, work=work)
    torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"target": "done", "chunk": plan.chunk, "precision": precision, "n": n, "b": b}), flush=True)


def summary_name(precision: str, n: int, b: int) -> str:
    """Base name (under profiles/) of the traffic summary of one workload."""
    return f"apply_{precision}_{n}{'_period3' if b == 3 else ''}_traffic"


def _read(d: str, counter: str) -> dict:
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    acc: dict[str, list[float]] = {}
    for f in files:
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "")
            acc.setdefault(name, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _workload(d: str) -> dict:
    """The target run's line (log next to the counter directory): densities per apply dispatch and
    the plan's precision, n and b."""
    with open(d.rstrip("/") + ".log") as fh:
        for line in fh:
            if line.startswith("{") and '"target"' in line:
                w = json.loads(line)
                return dict(chunk=int(w["chunk"]), precision=w.get("precision", "fp64"), n=int(w.get("n", 2048)),
                            b=int(w.get("b", 2)))
    raise RuntimeError(f"no target line in {d}.log")


def summarise(fetch_dir: str, write_dir: str, out: str) -> dict:
    fetch = _read(fetch_dir, "FETCH_SIZE")
    write = _read(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copy" in k.lower() or "elementwise" in k.lower()]
    if not copy:
        raise RuntimeError("calibration copy kernel not found in the counters")
    ck = max(copy, key=lambda k: fetch[k])
    f_scale = COPY_BYTES / (fetch[ck] * 1024.0)
    w_scale = COPY_BYTES / (write[ck] * 1024.0)
    kernels = {}
    for k in fetch:
        if not k.startswith("ws::k_"):
            continue
        kernels[k] = dict(fetch_kib=fetch[k], write_kib=write.get(k, 0.0),
                          read_bytes=fetch[k] * 1024.0 * f_scale,
                          write_bytes=write.get(k, 0.0) * 1024.0 * w_scale)
        kernels[k]["traffic_bytes"] = kernels[k]["read_bytes"] + kernels[k]["write_bytes"]
    wl = _workload(fetch_dir)
    chunk = wl["chunk"]
    prec, n, b = wl["precision"], wl["n"], wl["b"]
    res = dict(source_hash=source_hash(), densities_per_dispatch=chunk, calibration_kernel=ck, fetch_scale=f_scale,
               write_scale=w_scale, copy_bytes=COPY_BYTES, precision=prec, n=n, b=b,
               workload=f"{prec.upper()} log|x| plan, n={n}, b={b}, two chunks of {chunk} densities "
                        f"(per-dispatch averages)",
               kernels=kernels)
    opts = f" --precision {prec} --n {n} --b {b}"
    with open(out + ".json", "w") as fh:
        json.dump(res, fh, indent=1)
    lines = [f"# HBM traffic per dispatch, {prec.upper()} apply at n={n}, period b={b} (rocprofv3 PMC)", "",
             "Commands ($R: the repository root; $OUT: an output folder):", "", "```",
             "cd /tmp && export TMPDIR=/tmp",
             "rocprofv3 --pmc FETCH_SIZE -d $OUT/pmc_fetch -o p --output-format csv -- "
             f"python3 $R/paper_2107_03958_amd/traffic.py target{opts} > $OUT/pmc_fetch.log",
             "rocprofv3 --pmc WRITE_SIZE -d $OUT/pmc_write -o p --output-format csv -- "
             f"python3 $R/paper_2107_03958_amd/traffic.py target{opts} > $OUT/pmc_write.log",
             "cd $R && python3 paper_2107_03958_amd/traffic.py summarise $OUT/pmc_fetch $OUT/pmc_write "
             f"profiles/{summary_name(prec, n, b)}", "```", "",
             f"Each apply dispatch covers {res['densities_per_dispatch']} densities.", "",
             f"Calibration: `{ck}` copying {COPY_BYTES >> 20} MiB read FETCH_SIZE {fetch[ck]:.0f} KiB "
             f"(scale {f_scale:.3f}) and WRITE_SIZE {write[ck]:.0f} KiB (scale {w_scale:.3f}).", "",
             "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | read (MB) | written (MB) |", "|---|---|---|---|---|"]
    for k, v in kernels.items():
        lines.append(f"| `{k}` | {v['fetch_kib']:.0f} | {v['write_kib']:.0f} | {v['read_bytes'] / 1e6:.1f} | "
                     f"{v['write_bytes'] / 1e6:.1f} |")
    lines += ["", f"Kernel source hash: `{res['source_hash']}`."]
    with open(out + ".md", "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return res


# Pass of each apply-kernel kind (the second template argument of ws::k_pass1).
PASS_OF_KIND = {"0": "forward row pass (k_rows_fwd_real)", "1": "column pass (k_cols)",
                "3": "inverse row pass (k_rows_inv_real)"}


def stats_summary(stats_csv: str, out_md: str, title: str, command: str, pattern: str = "") -> list:
    """Markdown table of the ws:: kernels whose name matches the regular expression `pattern`
    (all of them when empty) in a rocprofv3 kernel_stats.csv, sorted by total time; returns the rows."""
    import re
    rows = []
    for r in csv.DictReader(open(stats_csv)):
        name = r["Name"].split("(")[0].replace("void ", "")
        if not name.startswith("ws::") or (pattern and not re.search(pattern, name)):
            continue
        kind = ""
        if name.startswith("ws::k_pass1<"):
            kind = PASS_OF_KIND.get(name.split(",")[1].strip(), "")
        rows.append(dict(name=name, kind=kind, calls=int(r["Calls"]), avg_us=float(r["AverageNs"]) / 1e3,
                         min_us=float(r["MinNs"]) / 1e3, max_us=float(r["MaxNs"]) / 1e3,
                         share=float(r["Percentage"])))
    rows.sort(key=lambda x: -x["share"])
    lines = [f"# {title}", "", "Command ($R: the repository root; $OUT: an output folder):", "", "```",
             "cd /tmp && export TMPDIR=/tmp", command, "```", "",
             "| kernel | pass | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|---|"]
    for x in rows:
        lines.append(f"| `{x['name']}` | {x['kind']} | {x['calls']} | {x['avg_us']:.1f} | {x['min_us']:.1f} | "
                     f"{x['max_us']:.1f} | {x['share']:.1f}% |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return rows


def load_for_current_sources(path: str):
    """The stored traffic summary if it was taken with the current kernel sources, else None."""
    try:
        with open(path) as fh:
            res = json.load(fh)
    except (OSError, ValueError):
        return None
    return res if res.get("source_hash") == source_hash() else None


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "target":
        import argparse
        ap = argparse.ArgumentParser()
        ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
        ap.add_argument("--n", type=int, default=2048)
        ap.add_argument("--b", type=int, default=2)
        a = ap.parse_args(sys.argv[2:])
        target(a.precision, a.n, a.b)
    elif len(sys.argv) in (6, 7) and sys.argv[1] == "stats":
        stats_summary(*sys.argv[2:])
    elif len(sys.argv) == 5 and sys.argv[1] == "summarise":
        print(json.dumps(summarise(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
    else:
        print(__doc__)
        sys.exit(2)
