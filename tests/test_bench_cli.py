"""bench.py's command line on the CPU: more than one GPU is refused with a
message (the library has no multi-GPU path), and the help names every option
the benchmark's documented runs use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_options():
    r = run("--help")
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--workload", "--path", "--mode", "--seed-filter", "--streams",
                "--launch", "--raw", "--kalman", "--extrapolate", "--calib-copy-mib", "--no-cpu-baseline"):
        assert opt in r.stdout, opt
