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


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_admission_policy_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    # the same scenarios in a host build with AddressSanitizer and UBSan: no
    # out-of-bounds access, use after free, leak or undefined behaviour
    exe = tmp_path / "serve_policy_test_san"
    src = os.path.join(ROOT, "tests", "serve_policy_test.cpp")
    inc = os.path.join(ROOT, "paper_1803_02132_amd", "csrc")
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    try:
        subprocess.run(["g++", "-std=c++17", "-Wall", *flags, "-I", inc, src, "-o", str(exe)], check=True,
                       capture_output=True, text=True)
    except subprocess.CalledProcessError as e:
        pytest.skip("no sanitizer runtime for g++ here: " + e.stderr[-200:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().startswith("ok")
