"""Compile the CPU oracle (plain C) into ``oracle/libfwrs_oracle.so``.

Test infrastructure: the tests, the smoke check and the benchmark's CPU
baseline load the result; the product path never does.

Flags: binary32 arithmetic one operation at a time (no contraction into fused
multiply-adds, no fast-math reassociation, SSE rather than x87 registers), so
every rounding the oracle performs is the IEEE one its source spells out.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fwrs_oracle.c")
LIB = os.path.join(HERE, "libfwrs_oracle.so")

CFLAGS = [
    "-O2", "-std=c11", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
    "-mfpmath=sse", "-msse2", "-fno-unsafe-math-optimizations",
    "-Wall", "-Wextra",
]


def build(force: bool = True, extra_flags: list[str] | None = None, out: str | None = None) -> str:
    """Build the oracle library; returns its path.  ``extra_flags`` and ``out``
    let a test build a variant (for example with a planted mistake) elsewhere."""
    target = out or LIB
    if not force and os.path.exists(target) and os.path.getmtime(target) >= os.path.getmtime(SRC):
        return target
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), "-o", target, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return target


if __name__ == "__main__":
    print(build(force=True))
    sys.exit(0)
