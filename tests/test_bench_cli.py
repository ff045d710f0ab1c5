"""bench.py's command line on the CPU: one GPU only, and argument checks that run before
any GPU work."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_workload_options():
    r = _run("--help")
    assert r.returncode == 0
    for opt in ("--config", "--prec", "--approx", "--adjoint", "--graph", "--cross", "--exclude-self",
                "--shard", "--nside", "--m-max", "--cpu-sample"):
        assert opt in r.stdout, opt
