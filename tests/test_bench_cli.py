"""bench.py's command line on a host without a GPU: several GPUs are refused with a message
(the path runs on one GPU), before any device work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_help_lists_the_legs():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                         capture_output=True, text=True, timeout=300)
    assert out.returncode == 0
    for flag in ("--steps", "--warmup", "--main-only", "--serve-batch", "--no-fp64"):
        assert flag in out.stdout, flag
