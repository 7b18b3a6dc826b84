"""The benchmark's command line without a GPU: one GPU only (more exit with
a message), and its switches parse."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_switches():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--no-cpu", "--no-plain", "--no-soft",
                 "--no-window", "--no-stress", "--no-template", "--no-table1",
                 "--no-volume",
                 "--tune-cache", "--no-autotune", "--copy-gib"):
        assert flag in r.stdout, flag
