"""The serving path's host copy pool (csrc/host_copy.h), built for the host with g++.

Several threads copy pieces of random sizes through one pool at once; every
byte must arrive, and the float check made while copying must flag exactly the
copies that hold a planted negative or non-finite value in a checked piece.  A
second build runs under ThreadSanitizer (host code only).
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1206_6468_amd", "csrc")
SRC = os.path.join(HERE, "native", "host_copy_check.cpp")


def _build(tmp_path, name, extra):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O2", "-pthread", *extra, "-I", CSRC, SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    return exe


def test_copy_pool_concurrent_callers(tmp_path):
    exe = _build(tmp_path, "hc", [])
    r = subprocess.run([exe, "4", "40"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr


def test_copy_pool_under_thread_sanitizer(tmp_path):
    exe = _build(tmp_path, "hc_tsan", ["-fsanitize=thread", "-g"])
    r = subprocess.run([exe, "3", "6"], capture_output=True, text=True, timeout=600)
    if "FATAL: ThreadSanitizer: unexpected memory mapping" in r.stderr:
        pytest.skip("ThreadSanitizer cannot map its shadow memory on this kernel")
    assert r.returncode == 0 and "WARNING: ThreadSanitizer" not in r.stderr, r.stdout + r.stderr[-3000:]
