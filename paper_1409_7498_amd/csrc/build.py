"""Build ``libpolyreact.so`` (HIP for gfx950) in-tree with hipcc.

Flags: -O3, FP contraction off (the distance contract rounds every FP32
operation on its own), packed-FP32 instructions disabled, gfx950 only.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libpolyreact.so")
SOURCES = ["kernels.hip", "api.hip", "logsort.hip"]
HEADERS = ["common.hpp", os.path.join("..", "..", "include", "polyreact.h")]

HIPFLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
            "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(out=LIB, verbose=False):
    objs = []
    tmpdir = os.path.join(HERE, "_build")
    os.makedirs(tmpdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(tmpdir, src + ".o")
        cmd = [hipcc(), *HIPFLAGS, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run([hipcc(), "-shared", "--offload-arch=gfx950", *objs, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
