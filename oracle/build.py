"""Compile the CPU oracle (``sad_oracle.c``) into ``liboracle_sad.so`` beside it.

Test infrastructure: the oracle is the plain C reference the GPU library is checked
against.  Built with gcc, no contraction of multiply-add, no fast-math, so every
float32 operation in the canonical score is a single correctly rounded IEEE op.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sad_oracle.c")
LIB = os.path.join(HERE, "liboracle_sad.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-frounding-math", "-fno-strict-aliasing", "-fopenmp", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    """Compile the oracle library; return its path."""
    cmd = ["gcc", *CFLAGS, "-o", LIB + ".tmp", SRC, "-lm", "-lgomp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
