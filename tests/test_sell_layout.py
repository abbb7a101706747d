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


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_sell_layout_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The same host code and checks built with AddressSanitizer and
    UndefinedBehaviorSanitizer (host code only, g++; any report aborts)."""
    exe = tmp_path / "sell_check_san"
    src = [os.path.join(ROOT, "tests", "sell_layout_check.cpp"),
           os.path.join(ROOT, "paper_2103_00736_amd", "csrc", "acs_problem.cpp")]
    flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    subprocess.run(["g++", *flags, "-o", str(exe)] + src, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    print(out.stdout[-2000:])
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr[-4000:]
    assert out.stdout.strip().endswith("ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_sell_layout_under_thread_sanitizer(tmp_path):
    """The layouts of large problems are built on several host threads (each
    writing only the rows, columns or entries it owns): the same checks built
    with ThreadSanitizer (host code only, g++; any data race aborts)."""
    exe = tmp_path / "sell_check_tsan"
    src = [os.path.join(ROOT, "tests", "sell_layout_check.cpp"),
           os.path.join(ROOT, "paper_2103_00736_amd", "csrc", "acs_problem.cpp")]
    flags = ["-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=thread", "-pthread"]
    subprocess.run(["g++", *flags, "-o", str(exe)] + src, check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:abort_on_error=0")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=900, env=env)
    print(out.stdout[-2000:])
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert "ThreadSanitizer" not in out.stderr, out.stderr[-4000:]
    assert out.stdout.strip().endswith("ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_layouts_do_not_depend_on_the_number_of_host_threads(tmp_path):
    """Problem creation and the layouts of large problems are split over host
    threads (at most ACS_HOST_THREADS): one thread and several must build the
    same arrays, bit for bit."""
    exe = tmp_path / "sell_check_threads"
    src = [os.path.join(ROOT, "tests", "sell_layout_check.cpp"),
           os.path.join(ROOT, "paper_2103_00736_amd", "csrc", "acs_problem.cpp")]
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-o", str(exe)] + src, check=True)
    hashes = {}
    for threads in ("1", "3", "8"):
        out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                             env=dict(os.environ, ACS_HOST_THREADS=threads))
        assert out.returncode == 0, out.stdout + out.stderr
        hashes[threads] = [l for l in out.stdout.splitlines() if l.startswith("hash ")]
        assert len(hashes[threads]) == 5, out.stdout
    assert hashes["1"] == hashes["3"] == hashes["8"], hashes
