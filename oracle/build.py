"""Build the C oracle (test infrastructure only) into ``oracle/liboracle.so``.

Compiled with gcc, ``-ffp-contract=off`` so that no multiply-add is fused and
every product is rounded before it is added, OpenMP for threads, and a
portable x86-64-v3 target so the same shared object runs on any AVX2 host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ata_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
