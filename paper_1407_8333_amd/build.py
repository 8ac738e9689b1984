"""Build the gfx950 frequency-Hough shared library in-tree.

    python -m paper_1407_8333_amd.build

Produces paper_1407_8333_amd/libfh.so from csrc/*.hip and csrc/*.cpp with
hipcc.  Floating-point contraction is off so that the fixed-point stripe
edges follow the IEEE definition exactly; packed FP32 instructions are
disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfh.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["fh_kernels.hip", "fh_runtime.cpp"]
# LDS-atomic microbenchmark used by the benchmark for the tile kernel's roof
PROBE_SOURCES = ["fh_probe.hip"]
PROBE_LIB = os.path.join(HERE, "libfh_probe.so")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep single-lane atomics as issued (the tile scheduler claims its next
    # tile with an atomic whose result is only needed when the tile ends)
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function",
]


def _hipcc(sources, out, verbose):
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-x", "hip", *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building %s" % os.path.basename(out))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _hipcc(SOURCES, LIB, verbose)
    _hipcc(PROBE_SOURCES, PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
