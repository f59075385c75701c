"""CPU test of the request server's admission policy (serve_policy.h), compiled
with g++ into a small host program: FIFO order, footprint back-pressure,
rejection of requests larger than the budget, resident-slot limits, bounded
overtaking of a blocked head and absence of starvation."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy(tmp_path):
    exe = tmp_path / "admission_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                           "-I" + os.path.join(ROOT, "paper_2512_04216_amd", "csrc"),
                           os.path.join(ROOT, "tests", "cpp", "admission_test.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all checks passed" in out.stdout
