"""Command-line contract of bench.py that holds without a GPU: one GPU only,
and the flags the serving measurement adds."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*argv):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_help_lists_streams_flag():
    r = run_bench("--help")
    assert r.returncode == 0
    assert "--streams" in r.stdout and "--gpus" in r.stdout
