"""Compile the HIP library ``libdd.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdd.so")
SOURCES = ["plan.cpp", "api.cpp", "tune.cpp", "batch.cpp", "survey.cpp", "fwd_int.hip", "fwd_direct.hip", "kernels_f32.hip", "bin.hip", "corner.hip", "noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # never emit packed FP32 arithmetic (v_pk_add/mul/fma_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep single-lane atomics plain: the wave-level atomic rewrite waits for the
    # result at once, which would expose the batched kernel's claim-ahead latency
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall",
]


def build(verbose: bool = False) -> str:
    """Always recompile libdd.so from csrc/ (a few tens of seconds)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *HIPCC_FLAGS, *srcs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
