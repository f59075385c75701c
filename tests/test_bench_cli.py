"""Host checks of bench.py's command line: more than one GPU is refused with a
message and exit status 2 before anything touches a device, and every
workload the help lists is accepted by the parser."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workloads():
    r = _bench("--help")
    assert r.returncode == 0
    for name in ("28q", "small", "fused", "fused_mfma", "qaoa", "serving", "cost", "pblock", "sampling",
                 "midcircuit"):
        assert name in r.stdout
