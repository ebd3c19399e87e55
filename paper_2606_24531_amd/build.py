"""Builds libaceseek.so (gfx950) in-tree with hipcc, and beside it
libacecalib.so, the calibration kernels bench.py times (not linked into the
decode library)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaceseek.so")
SOURCES = ["host.cpp", "encoder.cpp", "kernels.hip"]
CALIB_LIB = os.path.join(HERE, "libacecalib.so")
ARCH = os.environ.get("ACESEEK_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmd = ["hipcc", "-c", "-O3", "-std=c++17", "-fPIC", "-Wall",
               "--offload-arch=" + ARCH,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-x", "hip", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH, "-pthread", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # calibration library: one file, built as its own shared object
    tmp = CALIB_LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", "-O3", "-std=c++17", "-Wall", "--offload-arch=" + ARCH,
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-x", "hip", os.path.join(CSRC, "calib.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CALIB_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
