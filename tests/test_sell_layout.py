"""Host logic of the CG's data layout, without a GPU: the row renumbering and
the SELL layouts built by the library's problem code (compiled here with g++
from paper_2103_00736_amd/csrc/acs_problem.cpp).  The check program replays
the GPU kernels' task decomposition on the CPU and compares both products
with plain CSR sums (power-law rows, rows at every task-kind boundary, a
dense column, a single row, an empty matrix)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_sell_layout_and_row_renumbering(tmp_path):
    exe = tmp_path / "sell_check"
    src = [os.path.join(ROOT, "tests", "sell_layout_check.cpp"),
           os.path.join(ROOT, "paper_2103_00736_amd", "csrc", "acs_problem.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe)] + src, check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
