"""Build the FP64 CPU oracle library ``liboracle.so`` (test infrastructure).

The oracle is compiled with gcc, contraction of a*b+c into fused multiply-adds
off and no fast-math, so that its arithmetic is plain IEEE binary64 with
correctly rounded division and square root.  OpenMP parallelises the outer
loop of each stage and does not change any result.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hydro_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
OPC_SRC = os.path.join(HERE, "opcount.cpp")
OPC_LIB = os.path.join(HERE, "libopcount.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
          "-shared", "-fPIC", "-Wall"]


def _stale(lib, srcs):
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(s) for s in srcs)


def build(force: bool = True) -> str:
    """Compile the oracle (and its operation-counting variant); returns the
    path of the oracle library."""
    hdr = os.path.join(HERE, "hydro_oracle.h")
    if force or _stale(LIB, [SRC, hdr]):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"], check=True)
        os.replace(tmp, LIB)
    if force or _stale(OPC_LIB, [SRC, hdr, OPC_SRC]):
        tmp = OPC_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["g++", "-O1", "-ffp-contract=off", "-std=c++17", "-fPIC", "-shared",
                        "-w", "-o", tmp, OPC_SRC], check=True)
        os.replace(tmp, OPC_LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
