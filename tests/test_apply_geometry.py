"""Tile geometry of the apply kernels checked on the host (no GPU): see
tests/apply_geometry_check.cpp.  Compiled with hipcc, run on the CPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(_hipcc() is None, reason="needs hipcc")
def test_apply_geometry(tmp_path):
    exe = tmp_path / "apply_geometry_check"
    cmd = [_hipcc(), "-std=c++17", "--offload-arch=gfx950", "-O1", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "apply_geometry_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    assert "passed" in res.stdout
