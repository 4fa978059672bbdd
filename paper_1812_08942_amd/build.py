"""Builds libgraphreduce.so (the HIP/C-ABI library) in-tree with hipcc for
gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgraphreduce.so")
SOURCES = ["gr_prims.hip", "gr_phase_a.hip", "gr_affinity.hip", "gr_aggregate.hip", "gr_restrict.hip", "gr_autograd.hip",
           "gr_sgd.hip", "gr_eigen.hip", "gr_api.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # no packed fp32 instructions (v_pk_*_f32) anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(force: bool = True, verbose: bool = False) -> str:
    deps = sources() + [os.path.join(CSRC, "gr_internal.hpp"),
                        os.path.join(CSRC, "gr_device.hpp"),
                        os.path.join(INCLUDE, "graphreduce.h")]
    if not force and os.path.exists(LIB) and \
            os.path.getmtime(LIB) >= max(os.path.getmtime(d) for d in deps):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", INCLUDE, "-I", CSRC, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--lazy" not in sys.argv, verbose=True))
