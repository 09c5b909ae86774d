"""Host-side logic of the serving engine (arena allocator, admission, batching),
built from serve_core.hpp with g++ under AddressSanitizer/UBSan; no GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_serve_core(tmp_path):
    exe = tmp_path / "serve_core_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           os.path.join(HERE, "serve_core_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert "passed" in res.stdout
