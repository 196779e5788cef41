"""Host-side checks of the serving loop's policy (HBM pool allocator and the
choice of the next request to admit), compiled from the library's own header
with g++: no GPU involved."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_serve_policy(tmp_path):
    exe = tmp_path / "serve_policy_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1601_04280_amd", "csrc"),
                    os.path.join(HERE, "serve_policy_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
