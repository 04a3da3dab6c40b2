"""Build libcgs.so (gfx950) from the HIP sources with hipcc, in-tree.

Flags: -O3 for gfx950; packed-FP32 instruction selection disabled (plain
FP32 VALU ops only); default IEEE single-precision division and square root
(the tile skeleton relies on correctly rounded results); no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "sort.hip", "render_fwd.hip", "render_bwd.hip", "train.hip", "mh.hip"]
LIB = os.path.join(HERE, "libcgs.so")
ARCH = os.environ.get("CGS_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out: str, extra=()):
    return (["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wl,-z,defs", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", out]
            + list(extra) + [os.path.join(CSRC, s) for s in SOURCES])


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
