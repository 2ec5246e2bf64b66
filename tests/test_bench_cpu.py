"""CPU tests of bench.py's contract that need no GPU: it measures one GPU
and exits with a message for any other count, before touching a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    for n in ("2", "8"):
        r = run("--gpus", n)
        assert r.returncode == 2, r
        assert "one GPU only" in r.stderr and f"asked for {n}" in r.stderr
        assert r.stdout == ""


def test_help_lists_the_legs():
    r = run("--help")
    assert r.returncode == 0
    for leg in ("main", "batch", "serve", "snapshots", "adaptive", "large"):
        assert leg in r.stdout
