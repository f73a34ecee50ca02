"""Host checks of the server's admission policy (no GPU): the C++ policy that
tsb_server_* applies, compiled with g++ against named scenarios (among them a
geometry whose idle workspace must grow while other geometries' idle
workspaces hold the memory) and random ones checked against its invariants
(a request never waits while nothing runs; releases and slots respect the
budget)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_admission_policy(tmp_path):
    exe = tmp_path / "serve_policy_test"
    src = os.path.join(ROOT, "tests", "serve_policy_test.cpp")
    inc = os.path.join(ROOT, "paper_1803_02132_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", inc, src, "-o", str(exe)], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().startswith("ok")
