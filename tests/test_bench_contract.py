"""Host-side checks of bench.py's command line: one GPU only, and every
workload listed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=300)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_workloads_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("helmholtz_cubes_n64", "uneven_mix_bf16", "helmholtz_cubes_n128_lsq",
              "helmholtz_cubes_n512_paper"):
        assert w in r.stdout
