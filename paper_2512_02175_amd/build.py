"""Builds libmetricgraph.so (the C ABI of include/metricgraph.h) for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("mg_api.hip", "mg_kernels.hip", "mg_calib.hip")]
LIB = os.path.join(HERE, "libmetricgraph.so")
ARCH = os.environ.get("MG_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # the FP64 path must evaluate exactly the operations it writes
    "-ffp-contract=off",
    # no packed FP32 arithmetic on this target
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(extra: list[str] | None = None, out: str = LIB) -> str:
    """Compiles every source (always; the call is the build check)."""
    tmp = out + ".tmp"
    cmd = ["hipcc", *FLAGS, *(extra or []), "-o", tmp, *SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1:]))
