"""Compile the CPU oracle (test infrastructure) into oracle/libhrr_oracle.so.

Plain gcc, binary32 arithmetic rounded operation by operation: no FMA
contraction, SSE math (never x87 extended precision), no fast-math.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hrr_oracle.c")
OUT = os.path.join(HERE, "libhrr_oracle.so")

FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
         "-fno-fast-math", "-msse2", "-mfpmath=sse", "-fvisibility=hidden",
         "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = ["gcc", *FLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
