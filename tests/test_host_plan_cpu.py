"""The solver's host-side planning (argument checks, offsets, extents,
host-resident copy runs, memory-limited chunk capacity) compiled for the CPU
with AddressSanitizer and UndefinedBehaviorSanitizer and run on random and
invalid batches, and with ThreadSanitizer planning batches on four threads at
once, one planner per thread as with one handle per thread (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_plan_under_sanitizers(tmp_path):
    exe = tmp_path / "host_plan_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.join(ROOT, "paper_1609_08114_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host_plan_check.cpp"), "-o", str(exe)])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_plan_threads_under_tsan(tmp_path):
    exe = tmp_path / "host_plan_threads"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=thread",
                           "-pthread", "-I", os.path.join(ROOT, "paper_1609_08114_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host_plan_check.cpp"), "-o", str(exe)])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe), "threads"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "0 failures" in r.stdout
