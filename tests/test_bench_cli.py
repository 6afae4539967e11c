"""The command-line contract of bench.py that needs no GPU: one GPU only (--gpus N > 1 exits with
status 2 and says why, before touching a device), and the precision is one the library has."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_precision_is_refused():
    r = _run("--precision", "fp8")
    assert r.returncode == 2 and "invalid choice" in r.stderr
