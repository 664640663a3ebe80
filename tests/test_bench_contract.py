"""bench.py's command line: one GPU only, and the options the measurement uses."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_options():
    r = _bench("--help")
    assert r.returncode == 0
    for opt in ("--steps", "--warmup", "--no-cpu", "--no-forms", "--forms", "--calibrate"):
        assert opt in r.stdout
