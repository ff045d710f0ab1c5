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


def test_entry_errors_one_map_and_several_maps():
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    rng = np.random.default_rng(0)
    ref = rng.normal(size=(3, 5, 4, 4)) + 1j * rng.normal(size=(3, 5, 4, 4))
    ref = ref + np.conj(np.swapaxes(ref, -1, -2))  # Hermitian per m, like zeta_m
    test = ref * (1 + 1e-7 * rng.normal(size=ref.shape))
    one = bench.entry_errors(test[1], ref[1])
    many = bench.entry_errors(test, ref)
    assert many["entries"] == 3 * one["entries"]
    assert one["max_rel_err"] <= many["max_rel_err"] < 1e-6
    assert len(many["max_rel_err_per_m"]) == 5 and "map" in many["worst"][0]
    assert "map" not in one["worst"][0]


def test_fftlog_option_is_listed():
    r = _run("--help")
    assert "--fftlog" in r.stdout and "--hist" in r.stdout
