"""bench.py's argument checks run before any GPU work (no GPU needed): the
engine has one GPU per run, and a run needs at least one timed step."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_zero_steps_rejected():
    r = _run("--steps", "0")
    assert r.returncode == 2
    assert "--steps" in r.stderr
