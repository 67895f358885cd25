"""CPU test of the serving runtime's host bookkeeping (first-fit pool, admission step), built from
csrc/host_pool.h with the host compiler under AddressSanitizer and UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2110_12065_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pool_and_admission_under_sanitizers(tmp_path):
    exe = tmp_path / "host_runtime_check"
    src = os.path.join(ROOT, "tests", "host_runtime_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", f"-I{CSRC}", src, "-o", str(exe)], check=True, timeout=300)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host runtime checks passed" in r.stdout
