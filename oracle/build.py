"""Build step for the CPU oracle (test infrastructure): gcc -> oracle/_fd_oracle.so.

The oracle is plain C99 + OpenMP compiled for generic x86-64 (no -march=native:
the shared object is built once and also runs on other hosts), with FMA
contraction off so that every product and sum rounds as written.

A second copy of the same source, oracle/_fd_oracle_fast.so, is compiled with
-O3 for x86-64-v3 (AVX2, the level every current server CPU has) for the
benchmark's CPU baseline only; the code is the same, FMA contraction stays off.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fd_oracle.c")
LIB = os.path.join(HERE, "_fd_oracle.so")
LIB_FAST = os.path.join(HERE, "_fd_oracle_fast.so")


def _one(out: str, opt: list, force: bool) -> str:
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=gnu11"] + opt + ["-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", SRC, "-o", tmp,
                                         "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True, fast: bool = False) -> str:
    """Build both copies (force: even when up to date); return the path of
    the one asked for."""
    a = _one(LIB, ["-O2"], force)
    b = _one(LIB_FAST, ["-O3", "-march=x86-64-v3"], force)
    return b if fast else a


if __name__ == "__main__":
    print(build())
