"""CPU tests of the serving scheduler (admission, back-pressure, errors,
failure propagation, concurrency) through a stand-in backend; see
tests/serve_harness.cpp.  The HIP backend is tested in test_gpu_serve.py."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("serve") / "harness")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-pthread",
                           "-fsanitize=address,undefined", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_1503_03492_amd", "csrc"),
                           os.path.join(ROOT, "tests", "serve_harness.cpp"), "-o", exe])
    return exe


@pytest.mark.parametrize("case", ["basic", "admission", "busy", "errors", "device_failure",
                                  "threads", "shutdown"])
def test_scheduler(harness, case):
    r = subprocess.run([harness, case], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert f"ok {case}" in r.stdout
