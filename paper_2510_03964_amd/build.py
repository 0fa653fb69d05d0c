"""Build the gfx950 HIP library ``libfwrs.so`` in-tree with hipcc.

Floating-point flags are part of the method's contract: no contraction into
fused multiply-adds (-ffp-contract=off), correctly rounded binary32 division
and square root, denormals kept, and no packed-FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfwrs.so")
SOURCES = [os.path.join(CSRC, "fwrs_kernels.hip"), os.path.join(CSRC, "fwrs_api.hip")]
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
DEPS = SOURCES + [os.path.join(CSRC, "fwrs_device.hpp"), os.path.join(CSRC, "fwrs_internal.hpp"),
                  os.path.join(os.path.dirname(HERE), "include", "fwrs.h")]

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", f"-I{INCLUDE}", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument", "-Wno-pass-failed",
]


def build(force: bool = True, out: str | None = None, extra: list[str] | None = None) -> str:
    target = out or LIB
    if not force and os.path.exists(target):
        newest = max(os.path.getmtime(p) for p in DEPS)
        if os.path.getmtime(target) >= newest:
            return target
    tmp = target + ".tmp"
    cmd = ["hipcc", *FLAGS, *(extra or []), "-o", tmp, *SOURCES]
    subprocess.run(cmd, check=True)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(force=True, extra=sys.argv[1:]))
