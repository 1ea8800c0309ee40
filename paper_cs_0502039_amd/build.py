"""Build libaca.so (HIP for gfx950) in-tree with hipcc.

Every floating-point operation of the arrival-time recipe must round on its own,
so device and host code are compiled with -ffp-contract=off and no reassociation
(-fno-fast-math); packed FP32 instructions are disabled.  -fno-honor-nans is the
one relaxation, and it applies to device code only: no value a kernel computes
can be a NaN (times are finite and positive, u lies in (0, 1), every divisor is
at least 1), and the flag lets the compiler drop the NaN-quieting it would
otherwise put in front of every binary64 min in the enabling tests; it allows
no other change to any result.  Host code keeps IEEE NaN semantics, because it
validates caller arguments that may well be NaN.
"""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_PATH = os.path.join(HERE, "libaca.so")
SOURCES = ("aca_api.hip", "aca_kernels.hip", "aca_visit_fast.hip", "aca_batch.hip",
           "aca_batch_api.hip", "aca_server_api.hip")
ARCH = os.environ.get("ACA_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: cannot build libaca.so")
    return exe


def build_command(out: str, extra=()) -> list[str]:
    return [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-ffp-contract=off", "-fno-fast-math", "-Xarch_device", "-fno-honor-nans",
            "-fvisibility=hidden",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"),
            *[os.path.join(CSRC, s) for s in SOURCES], "-o", out, *extra]


def build(verbose: bool = False) -> str:
    tmp = LIB_PATH + f".tmp{os.getpid()}"
    cmd = build_command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
