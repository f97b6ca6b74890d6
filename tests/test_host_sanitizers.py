"""The serving loop's host code under AddressSanitizer + UndefinedBehavior-
Sanitizer and under ThreadSanitizer, on the CPU.

server.hip is compiled with g++ as C++ against tests/host_sanitize/: a
stand-in for the HIP runtime calls it makes (device memory is host memory,
events complete on a simulated clock) and for the plan calls (workspaces of
the library's sizes, an exec whose output depends only on the request's
inputs).  The driver runs four submitting threads and a stats reader under
a budget that forces queueing and eviction, a reused plan whose points grow
under a tight budget (which stalled before the scheduler retired a slot's
old buffer and fell back to a new plan), forced allocation failures, and a
destroy with work still queued; every output and the memory accounting are
checked against what the stand-in allocated.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "host_sanitize")
SOURCES_CXX = [os.path.join(ROOT, "paper_2605_01313_amd", "csrc", "server.hip")]
SOURCES = [os.path.join(HERE, "stub_runtime.cpp"), os.path.join(HERE, "driver.cpp")]


def build_and_run(tmp_path, sanitize):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "driver")
    flags = [f"-fsanitize={sanitize}"] + (["-fno-sanitize-recover=undefined"] if "undefined" in sanitize else [])
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", *flags,
           "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2605_01313_amd", "csrc"),
           "-x", "c++", *SOURCES_CXX, "-x", "none", *SOURCES, "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
    assert "ERROR" not in r.stderr and "WARNING: ThreadSanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_server_scheduler_under_address_and_ub_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "address,undefined")
    assert "evicted" in out and "drained" in out


def test_server_scheduler_under_thread_sanitizer(tmp_path):
    out = build_and_run(tmp_path, "thread")
    assert "growing points" in out
