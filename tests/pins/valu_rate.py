"""Builds and runs tests/pins/valu_rate.hip (the non-packed fp32 vector-ALU issue-rate microbenchmark) and
prints its JSON line.  Needs a GPU; measurement infrastructure, no part of the library."""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def main() -> int:
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "valu_rate")
        subprocess.run(["hipcc", "--offload-arch=gfx950", "-O3", "-ffp-contract=off", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", "-o", exe, os.path.join(HERE, "valu_rate.hip")],
                       check=True, capture_output=True)
        return subprocess.run([exe]).returncode


if __name__ == "__main__":
    sys.exit(main())
