"""The benchmark's command line on the CPU: more than one GPU is refused with a
message (the block hierarchy is not sharded), before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_storage_is_rejected():
    r = _run("--storage", "f64")
    assert r.returncode == 2
    assert "invalid choice" in r.stderr
