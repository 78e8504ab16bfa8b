"""Build step for the CPU oracle (test infrastructure): gcc -> oracle/_fd_oracle.so.

The oracle is plain C99 + OpenMP compiled for generic x86-64 (no -march=native:
the shared object is built once and also runs on other hosts), with FMA
contraction off so that every product and sum rounds as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fd_oracle.c")
LIB = os.path.join(HERE, "_fd_oracle.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
