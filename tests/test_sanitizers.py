"""The oracle and the C-ABI host code under AddressSanitizer and UBSan (CPU).

Runs the oracle's pin tests, the host-formulation tests and the library's
export / argument-validation tests in a child process that preloads clang's
shared sanitizer runtime and loads the instrumented builds of both libraries
(oracle: clang++ -fsanitize=address,undefined; libvelo: the same flags on its
host code).  Any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = ["test_oracle_cluster.py", "test_oracle_find.py", "test_oracle_find_rules.py", "test_oracle_fit.py",
         "test_oracle_kalman.py", "test_oracle_decode.py", "test_oracle_mlp.py", "test_oracle_seed_filter.py",
         "test_oracle_extrapolate.py", "test_library.py", "test_host_formulation.py"]


def _stale(lib, srcs):
    return not os.path.exists(lib) or any(os.path.getmtime(lib) < os.path.getmtime(s) for s in srcs)


def test_oracle_and_abi_host_code_under_asan_ubsan():
    if os.environ.get("VELO_SANITIZE") == "1":
        pytest.skip("already running under the sanitizers")
    import oracle
    from paper_2412_05041_amd import build
    try:
        rt = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    oracle.build(sanitize=True)
    if _stale(build.SAN_LIB, build.sources()):
        build.build(sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, VELO_SANITIZE="1", VELO_ORACLE_SANITIZE="1",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    probe = ("import ctypes, oracle; from paper_2412_05041_amd import velo; "
             "assert hasattr(ctypes.CDLL(None), '__asan_init'); "
             "assert oracle.LIB.endswith('_san.so') and velo.LIB_PATH.endswith('_san.so'); print('instrumented')")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and "instrumented" in r.stdout, r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *[os.path.join("tests", t) for t in TESTS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error:" not in out, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
