"""The runtime's ring of work-list tables (csrc/table_ring.h), built for the host
with g++ and driven against simulated asynchronous streams: a slot is rewritten
only after every read of its old contents has completed on every stream, every
read is ordered after the write it reads, and a key still in the ring is reused
without a rewrite (tests/native/table_ring_check.cpp)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1206_6468_amd", "csrc")
SRC = os.path.join(HERE, "native", "table_ring_check.cpp")


def test_table_ring_against_simulated_streams(tmp_path):
    exe = str(tmp_path / "trc")
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-I", CSRC, SRC, "-o", exe], capture_output=True,
                       text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    r = subprocess.run([exe, "20000"], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
