"""Compiles the HIP library librtg.so for gfx950 (in place, next to this file)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("rtg_kernels.hip", "rtg_ssim.hip", "rtg_collision.hip", "rtg_abi.hip")]
HEADERS = [os.path.join(HERE, "csrc", "rtg_internal.h"),
           os.path.join(os.path.dirname(HERE), "include", "rtg.h")]
LIB = os.path.join(HERE, "librtg.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # contraction off: every fused multiply-add is written explicitly
    "-ffp-contract=off",
    # hardware float atomics for the backward's per-record accumulation
    "-munsafe-fp-atomics",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc", *FLAGS, "-o", LIB + ".tmp", *SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    if verbose:
        print(r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
