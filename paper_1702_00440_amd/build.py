"""Build of the gfx950 shared library libgravidy_hip.so (in-tree, next to this file).

hipcc cross-compiles for gfx950 without a GPU. Packed FP32 instructions are
disabled for the device code (-packed-fp32-ops feature off); the host pass
warns that it does not know the feature, which is harmless.

Floating-point contraction is off (-ffp-contract=off): every fused multiply-add
is an explicit fma() in the source, so the arithmetic of a device function is
fixed by its text and the same function gives bitwise the same results in
every kernel it is inlined into (a cluster alone and packed with others, for
example). With contraction left to the compiler, the choice of which product
to fuse can depend on the surrounding kernel.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgravidy_hip.so")
SOURCES = ["gd_kernels.hip", "gd_api.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libgravidy_hip.so; returns its path."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-command-line-argument",
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
