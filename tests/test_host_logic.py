"""Host-side logic of the library checked without a GPU: the eigensolver's
index helpers (tournament pairings, NaN-safe ordering) compiled with g++ from
the same header the kernels include."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_jacobi_index_logic(tmp_path):
    exe = tmp_path / "jacobi_order"
    src = os.path.join(ROOT, "tests", "cpp", "test_jacobi_order.cpp")
    inc = os.path.join(ROOT, "paper_2211_07894_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", f"-I{inc}", src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
