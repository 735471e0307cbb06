"""Builds the stream-ordering checker (test infrastructure, CPU only).

libhipstub.so: hip_stub.cpp, a host-only stand-in for the HIP runtime that
records every ordering operation.  libdlt_lanecheck.so: the library's own
object files (the ones libdlt.so is linked from, built by the package's
build step) linked against the stand-in instead of the HIP runtime, so the
launch sequences that run are exactly the product's."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")
PKG_BUILD = os.path.join(os.path.dirname(os.path.dirname(HERE)), "paper_1505_00354_amd", "_build")
OBJS = ["dlt_kernels.o", "dlt_plan.o", "dlt_api.o"]
STUB = os.path.join(BUILD, "libhipstub.so")
LIB = os.path.join(BUILD, "libdlt_lanecheck.so")


def build(force: bool = False) -> str:
    objs = [os.path.join(PKG_BUILD, o) for o in OBJS]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError(f"library objects not built ({missing}); run the package build first")
    os.makedirs(BUILD, exist_ok=True)
    src = os.path.join(HERE, "hip_stub.cpp")
    newest = max(os.path.getmtime(p) for p in objs + [src])
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= newest:
        return LIB
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", src, "-o", STUB], check=True)
    subprocess.run(["g++", "-shared", "-fPIC", "-o", LIB, *objs, "-L" + BUILD, "-lhipstub",
                    "-Wl,-rpath," + BUILD, "-Wl,--no-undefined"], check=True)
    return LIB


if __name__ == "__main__":
    print(build(force=True))
