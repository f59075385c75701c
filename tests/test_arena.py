"""CPU test of the device-memory sub-allocator (arena.cpp), compiled with g++
into a small host program: random alloc / alloc_high / grow / shrink / free
sequences against a shadow map (no overlap, exact accounting, alignment,
grow exactly when the next extent is free and large enough, coalescing)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena(tmp_path):
    exe = tmp_path / "arena_test"
    csrc = os.path.join(ROOT, "paper_2512_04216_amd", "csrc")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I" + csrc,
                           os.path.join(ROOT, "tests", "cpp", "arena_test.cpp"), os.path.join(csrc, "arena.cpp"),
                           "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all checks passed" in out.stdout
