"""Builds libs3r.so (all HIP kernels and the C ABI) for gfx950 with hipcc.

Usage: python -m paper_2503_08217_amd.build  (or build() from Python).
The library is written next to this file so it travels with the source tree.
"""

from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libs3r.so")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # every decision of the projection is taken in the written operation order
    "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    # hardware float atomics for gradient accumulation
    "-munsafe-fp-atomics",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # an atomic at a wave-uniform address stays one instruction: no kernel
    # here has contended uniform-address atomics, and the optimizer's per-lane
    # combining loop cost the raster backward's LDS slot update a dozen
    # instructions per blended entry
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
]


def build(verbose: bool = False) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    cmd = ["hipcc", *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
