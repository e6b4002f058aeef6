"""CPU checks of the benchmark's command line: more than one GPU is refused
with a message before any device work, and the help lists the workloads."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_help_lists_workloads():
    r = run("--help")
    assert r.returncode == 0
    for w in ("splash1024x512", "droplet4096", "splash3d", "fa_diagnostics"):
        assert w in r.stdout
