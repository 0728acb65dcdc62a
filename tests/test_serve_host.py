"""The serving scheduler's admission, batching-window, memory and failure
handling, on the host: tests/serve_host_test.cpp drives the scheduler core
(paper_2306_11148_amd/csrc/serve_core.cpp, the same source linked into
libmoa.so) through a fake device that fails launches, completion markers and
allocations on demand. Built with the host compiler, once plainly and once
under ThreadSanitizer (clang's; a race in the scheduler fails the run). No
GPU, no HIP runtime, no oracle."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRCS = [os.path.join(ROOT, "paper_2306_11148_amd", "csrc", "serve_core.cpp"),
        os.path.join(ROOT, "tests", "serve_host_test.cpp")]
INCS = ["-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2306_11148_amd", "csrc")]
CLANG = "/opt/rocm/llvm/bin/clang++"


def _build_and_run(tmp_path, compiler, extra, env=None):
    exe = str(tmp_path / "serve_host_test")
    res = subprocess.run([compiler, "-std=c++17", "-O1", "-g", "-Wall", "-pthread", *extra, *INCS, *SRCS,
                          "-o", exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    run = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    return run


def test_scheduler_on_a_fake_device(tmp_path):
    run = _build_and_run(tmp_path, shutil.which("g++") or "g++", [])
    assert run.returncode == 0, run.stdout + run.stderr
    assert "all ok" in run.stdout
    for name in ("pool_blocks", "synthetic_lifecycle", "device_error_on_completion", "launch_and_marker_failures",
                 "device_out_of_memory", "budget_and_fcfs", "release_frees_budget", "batching_window",
                 "ticket_errors", "pool_reserve"):
        assert f"ok {name}" in run.stdout


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ of the ROCm toolchain not present")
def test_scheduler_under_thread_sanitizer(tmp_path):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    run = _build_and_run(tmp_path, CLANG, ["-fsanitize=thread"], env=env)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "ThreadSanitizer" not in run.stderr
    assert "all ok" in run.stdout
