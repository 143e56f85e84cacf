"""The serving loop's host code (csrc/serve.hip: queue, admission, worker
threads, waits, cancellation, shutdown) built for the CPU against a host
stand-in of the HIP runtime and of the solver, and run from many threads under
the compiler's thread sanitizer and, separately, its address sanitizer. No GPU
is involved; the GPU tests cover the same code with the real solver."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
CSRC = os.path.join(ROOT, "paper_1607_00315_amd", "csrc")


def _build_and_run(tmp_path, sanitizer):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    # the serving loop's source, compiled as plain host C++
    src = tmp_path / "serve_host.cpp"
    shutil.copyfile(os.path.join(CSRC, "serve.hip"), src)
    exe = tmp_path / f"serve_{sanitizer}"
    flags = ["-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-fno-omit-frame-pointer",
             "-I", HERE, "-I", CSRC, "-I", os.path.join(ROOT, "include")]
    cmd = ["g++", *flags, str(src), os.path.join(HERE, "stub_solver.cpp"),
           os.path.join(HERE, "driver.cpp"), "-o", str(exe), "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-6000:]
    assert "WARNING: ThreadSanitizer" not in out and "ERROR: AddressSanitizer" not in out, out[-6000:]
    return out


def test_serving_threads_under_thread_sanitizer(tmp_path):
    out = _build_and_run(tmp_path, "thread")
    assert "resolved 180 of 180" in out


def test_serving_threads_under_address_sanitizer(tmp_path):
    out = _build_and_run(tmp_path, "address")
    assert "resolved 180 of 180" in out
