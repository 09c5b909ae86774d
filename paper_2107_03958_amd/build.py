"""Build libwsconv.so (HIP, gfx950) in-tree.

Usage: python -m paper_2107_03958_amd.build [--jobs N] [--debug]

Every .hip source under csrc/ is compiled with hipcc for gfx950 and linked
into paper_2107_03958_amd/libwsconv.so.  Packed FP32 instructions are
disabled for all device code.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwsconv.so")
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def common_flags(debug: bool) -> list[str]:
    return [
        "-std=c++17",
        f"--offload-arch={ARCH}",
        "-fPIC",
        "-O1" if debug else "-O3",
        "-Wall",
        "-Wno-unused-function",
        "-Wno-unused-variable",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(HERE, "..", "include"),
    ]


def _compile(src: str, obj: str, flags: list[str]) -> tuple[str, int, str]:
    cmd = [hipcc(), *flags, "-c", src, "-o", obj]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; drop that harmless notice.
    noise = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"
    err = "\n".join(l for l in proc.stderr.splitlines() if noise not in l)
    return src, proc.returncode, err


def build(jobs: int = 4, debug: bool = False, verbose: bool = False, out: str = LIB,
          defines: list[str] | None = None, build_dir: str = BUILD) -> str:
    """Compile every csrc/*.hip and link `out`; `defines` are NAME=VALUE tile overrides."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    flags = common_flags(debug) + [f"-D{d}" for d in (defines or [])]
    objs = []
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        futs = []
        for src in srcs:
            obj = os.path.join(build_dir, os.path.basename(src)[:-4] + ".o")
            objs.append(obj)
            futs.append(ex.submit(_compile, src, obj, flags))
        failed = False
        for fut in futs:
            src, rc, err = fut.result()
            if err.strip() and (rc != 0 or verbose):
                sys.stderr.write(f"--- {os.path.basename(src)}\n{err}\n")
            failed = failed or rc != 0
    if failed:
        raise RuntimeError("HIP compilation failed")
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lrocblas"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, out)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--out", default=LIB, help="output library path")
    ap.add_argument("--build-dir", default=BUILD)
    ap.add_argument("-D", dest="defines", action="append", default=[], help="tile override NAME=VALUE")
    args = ap.parse_args(argv)
    print(build(args.jobs, args.debug, args.verbose, args.out, args.defines, args.build_dir))


if __name__ == "__main__":
    main()
