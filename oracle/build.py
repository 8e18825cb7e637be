"""Builds the FP64 CPU oracle (``oracle/liboracle.so``) with gcc.

Test infrastructure only: the product library never links this.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "oracle.c")]


def build(verbose: bool = False, src=None, out=None) -> str:
    """Compile oracle.c into liboracle.so (always recompiles).  `src` and
    `out` name another source file and library (the tests compile copies of
    the oracle with a deliberate mistake in them to show that the pins catch
    it); oracle/ stays on the include path for oracle.h."""
    srcs = SRC if src is None else [src]
    lib = LIB if out is None else out
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-I", HERE, "-o", tmp] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
