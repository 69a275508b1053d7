"""Compile the CPU oracle (plain C, double precision) into oracle/libsmki_oracle.so.

Test infrastructure only.  -ffp-contract=off and the absence of fast-math keep
the binary32 input contract (free-sample positions, voxel indices) bit exact:
every float operation is rounded on its own, with no fused multiply-add.
The default x86-64 target is used (no -march=native) so the library built
here also runs on another host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smki_oracle.c")
LIB = os.path.join(HERE, "libsmki_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
