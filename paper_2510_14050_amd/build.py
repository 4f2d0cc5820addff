"""Build libns.so for gfx950 with hipcc (cross-compiles without a GPU)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["ns_kernels.hip", "ns_api.hip"]
LIB = os.path.join(HERE, "libns.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
]


DEBUG_LIB = os.path.join(HERE, "libns_debug.so")


def build_library(verbose: bool = False) -> str:
    """libns.so, and libns_debug.so with every scatter / gather index of the
    radix passes and run scans checked against its bound (compiled side by side)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    jobs = []
    for out, extra in ((LIB, []), (DEBUG_LIB, ["-DNS_BOUNDS_CHECK=1"])):
        tmp = out + ".tmp"
        cmd = [HIPCC, *FLAGS, *extra, *srcs, "-o", tmp]
        jobs.append((out, tmp, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.PIPE, text=True)))
    for out, tmp, p in jobs:
        so, se = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(so + se)
            raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
        if verbose:
            sys.stderr.write(se)
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
