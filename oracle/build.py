"""Build the CPU reference library (test infrastructure only).

The reference is plain C compiled with gcc at -O2 and -ffp-contract=off, so
that every floating-point operation rounds as written.  It is never linked
into, loaded by, or called from the GPU library or its Python binding.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dlt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


FLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wextra"]


def compile_lib(src: str, out: str) -> None:
    """gcc with the flags above: src (a dlt_oracle.c beside its
    dlt_oracle_impl.h) -> shared library out."""
    subprocess.run(["gcc", *FLAGS, "-o", out, src], check=True, cwd=os.path.dirname(src))


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
        os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "dlt_oracle_impl.h"))
    ):
        return LIB
    compile_lib(SRC, LIB + ".tmp")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build())
