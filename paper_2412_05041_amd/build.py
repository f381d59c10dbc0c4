"""Builds libvelo.so (HIP, gfx950) in-tree with hipcc.

Device code is compiled without floating-point contraction (the track cuts
must evaluate exactly as written) and without packed FP32 instructions.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libvelo.so")
ARCH = os.environ.get("VELO_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


# Host code instrumented with AddressSanitizer and UBSan (each flag behind
# -Xarch_host: device code is built as usual); the process that loads the
# library must preload clang's shared sanitizer runtime.
SAN_LIB = os.path.join(HERE, "libvelo_san.so")
SAN_HOST = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -shared-libsan " \
           "-Xarch_host -fno-omit-frame-pointer -Xarch_host -g".split()


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


# The finder with per-phase wall-clock counters (a diagnostic build; slower).
PHASE_LIB = os.path.join(HERE, "libvelo_phase.so")


def build(verbose: bool = False, sanitize: bool = False, phase_timing: bool = False) -> str:
    lib = SAN_LIB if sanitize else (PHASE_LIB if phase_timing else LIB)
    tmp = lib + ".tmp%d" % os.getpid()
    flags = list(FLAGS)
    if phase_timing:
        flags.append("-DVELO_PHASE_TIMING")
    if sanitize:
        flags[flags.index("-O3")] = "-O1"
        flags += SAN_HOST
    cmd = ["hipcc", *flags, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def sanitizer_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime (to preload)."""
    import glob as g
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hits = sorted(g.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                      "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang's shared AddressSanitizer runtime was not found under " + rocm)
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv,
                phase_timing="--phase-timing" in sys.argv))
