"""Build libchaosvid.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2302_07411_amd.build

Flags: -ffp-contract=off and no fast-math keep every binary64 operation of
the chaotic maps a single correctly rounded IEEE operation (no FMA
contraction).  `-Xclang -target-feature -Xclang -packed-fp32-ops` turns off
the packed two-lane FP32 add/multiply/FMA instructions in the gfx950 device
pass (tests/test_build_flags.py compiles a float2 kernel with these flags and
checks that none is emitted, and that one is emitted without the flag); the
host pass does not know the feature, warns and ignores it.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libchaosvid.so")
ARCH = os.environ.get("CV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-Werror=infinite-recursion", "-Werror=return-type",
    "-Werror=uninitialized",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed to build libchaosvid.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
