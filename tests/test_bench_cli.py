"""bench.py's command line on the CPU: the options parse, and more than one GPU
is refused with a message (the benchmark runs on one GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_help_lists_workloads_and_options():
    r = run("--help")
    assert r.returncode == 0
    for opt in ("--workload", "--keep", "--subsets", "--reuse", "--windows", "--chunk", "--weighting",
                "--deblur-sizes"):
        assert opt in r.stdout
    for w in ("randomized", "deblur", "compare", "hbm_probe"):
        assert w in r.stdout


def test_more_than_one_gpu_is_refused():
    for extra in ([], ["--workload", "batch8"], ["--workload", "randomized"], ["--workload", "deblur"]):
        r = run("--gpus", "2", *extra)
        assert r.returncode == 2, (extra, r.stderr)
        assert "one GPU" in r.stderr
