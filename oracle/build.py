"""Build the CPU oracle (``oracle/oracle.c``) into ``oracle/liboracle.so``.

Test infrastructure only.  Flags: -O3, OpenMP, and -ffp-contract=off with no
fast-math, so that every FP32 operation of the distance test is rounded on its
own, as the arithmetic contract requires.  -fno-trapping-math only lets the
compiler evaluate both arms of the minimum-image select (no FP trap is ever
enabled here); rounding, operation order and contraction are unchanged, so the
tiled pair loop runs on SIMD lanes with the same per-pair results.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fno-trapping-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(out=LIB, extra=()):
    """Compile the oracle; ``extra`` adds -D flags (used by the mutation tests)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *extra, SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def ensure_built():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
