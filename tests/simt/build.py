"""Builds the library's kernel and host sources as x86 C++ against the host
stand-in of the HIP runtime in this folder (libaceseek_simt.so): a CPU build
for checks that need no GPU (lane-level execution of the kernels, array
bounds trapped).  Test infrastructure only; nothing in the product loads it."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2606_24531_amd", "csrc")
LIB = os.path.join(HERE, "libaceseek_simt.so")
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "host.cpp"),
           os.path.join(CSRC, "encoder.cpp"), os.path.join(HERE, "simt.cpp")]
CXX = "/opt/rocm/llvm/bin/clang++"

FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-I", HERE,
         "-DACE_GLOBAL=", "-DACE_OPAQUE(x)=((void)(x))",
         "-Wno-unknown-attributes", "-Wno-ignored-attributes",
         # out-of-bounds indexing of fixed-size arrays (the LDS tables) and
         # integer division by zero stop the process at the faulting access
         "-fsanitize=array-bounds,integer-divide-by-zero",
         "-fsanitize-trap=array-bounds,integer-divide-by-zero"]


def build(force: bool = False) -> str:
    deps = SOURCES + [os.path.join(HERE, "hip", "hip_runtime.h"), os.path.join(CSRC, "common.h")]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    objs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        subprocess.check_call([CXX, "-c", "-x", "c++"] + FLAGS + [src, "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([CXX, "-shared", "-pthread", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="-f" in sys.argv))
