"""CPU checks of bench.py's command line (no GPU work): more than one GPU is
refused with a message and a non-zero status before anything is imported
that touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_help_lists_the_legs():
    r = _run("--help")
    assert r.returncode == 0
    for leg in ("adjoint", "batch", "supercells", "marder", "deposit", "ablation"):
        assert leg in r.stdout
