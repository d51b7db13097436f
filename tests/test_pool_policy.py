"""Host-side rule for reusing solver workspaces (csrc/pool.h), compiled with g++.

A workspace whose solve ended with a reduction that gave up waiting, a tripped
host guard or an exception is freed instead of pooled, so stale partial sums in
its slots cannot reach the next solve.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1310_0956_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_pool_return_rule(tmp_path):
    exe = tmp_path / "pool_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-pthread", f"-I{CSRC}",
                    os.path.join(HERE, "native", "pool_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert "pool ok" in r.stdout
