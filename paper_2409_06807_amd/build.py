"""Build the gfx950 HIP library libkinopax.so in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkinopax.so")
SOURCES = [os.path.join(CSRC, f) for f in ("kp_kernels.hip", "kp_mlp.hip", "kp_api.hip")]
ARCH = os.environ.get("KP_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    # every expression compiles as written: the region estimates must round
    # exactly like their FP64 definition, so no implicit fused multiply-adds
    "-ffp-contract=off",
    # packed FP32 instructions stay off (toolchain correctness on this target)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # with packed FP32 off, the SLP vectorizer only packs booleans into
    # 16-bit lanes (compare, select 0/1, shift, bit-op) where a compare
    # into a lane mask and a scalar AND would do; off, the propagate kernel
    # needs fewer instructions and registers
    "-fno-slp-vectorize",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", *HIPCC_FLAGS,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
