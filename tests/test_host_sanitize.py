"""The library's multi-threaded host code under sanitizers, on the CPU: the
serving loop (server.cpp: lanes, admission, publication, submit / poll /
wait from several threads, replay, destroy with work queued) and the host
re-rank pool (host_rerank.cpp), built with clang's ThreadSanitizer, and once
with AddressSanitizer + UndefinedBehaviorSanitizer. The device side is
replaced by host stand-ins (tests/host_sanitize/fake_hip, fake_search.cpp):
"device" buffers are host memory and a search writes checkable results, so
the locking, condition variables and slot life cycle are what is exercised.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SRCS = [os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"),
        os.path.join(ROOT, "tests", "host_sanitize", "fake_search.cpp"),
        os.path.join(ROOT, "paper_2605_16007_amd", "csrc", "server.cpp"),
        os.path.join(ROOT, "paper_2605_16007_amd", "csrc", "host_rerank.cpp")]
INC = ["-I", os.path.join(ROOT, "tests", "host_sanitize", "fake_hip"), "-I", os.path.join(ROOT, "include"),
       "-I", os.path.join(ROOT, "paper_2605_16007_amd", "csrc")]


def _build(tmp_path, name, flags):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ of the ROCm toolchain not found")
    out = str(tmp_path / name)
    r = subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-pthread", *flags, *INC, *SRCS, "-o", out],
                       capture_output=True, text=True)
    if r.returncode != 0 and "cannot find" in r.stderr:
        pytest.skip("sanitizer runtime not available: " + r.stderr.strip()[:200])
    assert r.returncode == 0, r.stderr
    return out


def test_server_and_host_pool_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, "tsan_driver", ["-fsanitize=thread"])
    for run in range(5):  # races show up depending on the interleaving
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, TSAN_OPTIONS="halt_on_error=0"))
        assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.returncode == 0 and "0 failures" in r.stdout, (run, r.stdout, r.stderr[-2000:])


def test_server_and_host_pool_under_address_sanitizer(tmp_path):
    exe = _build(tmp_path, "asan_driver", ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "0 failures" in r.stdout, (r.stdout, r.stderr[-2000:])
