"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds none of the method's arithmetic: it only draws numbers.
Start blocks are N(0,1) from numpy's PCG64 generator, row-major D x n, as the
method's random initial search space; integer-valued blocks serve exact
(bit-for-bit) SpMMV comparisons; the model parameter sets are the workloads
the tests and the benchmark run.
"""
from __future__ import annotations

import numpy as np


def start_block(D: int, n: int, seed: int = 0) -> np.ndarray:
    """Row-major D x n block of standard normals (seeded)."""
    return np.random.default_rng(seed).standard_normal((D, n))


def int_block(D: int, n: int, seed: int = 0, bound: int = 1 << 10) -> np.ndarray:
    """Row-major D x n block of integers in [-bound, bound], as float64."""
    rng = np.random.default_rng(seed)
    return rng.integers(-bound, bound + 1, size=(D, n)).astype(np.float64)


# Workloads (sizes and parameters of the configurations that are measured).
HUBBARD8 = dict(model="hubbard", L=8, n_up=4, n_dn=4, t=1.0, U=4.0, periodic=True)
HUBBARD14 = dict(model="hubbard", L=14, n_up=7, n_dn=7, t=1.0, U=8.0, periodic=True)
ANDERSON200 = dict(model="anderson", L=200, t=1.0, W=16.5, seed=1)


def _splitmix64_uniforms(seed: int, n: int) -> list:
    """The first n outputs of SplitMix64(seed) as doubles in [0, 1) (top 53
    bits times 2^-53) -- the generator of the Anderson disorder, here only
    to draw instance parameters."""
    M = (1 << 64) - 1
    s = seed & M
    out = []
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & M
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        z ^= z >> 31
        out.append((z >> 11) * 2.0 ** -53)
    return out


def anderson_batch(seeds, L_lo: int = 20, L_span: int = 45, W_lo: float = 2.0, W_span: float = 18.0) -> list:
    """Batched Anderson workload: instance s draws L = L_lo + floor(L_span u0)
    and W = W_lo + W_span u1 from the first two outputs of SplitMix64(s); its
    disorder continues on the same stream (skip = 2).  The defaults give
    L in [20, 64], W in [2, 20)."""
    out = []
    for s in seeds:
        u0, u1 = _splitmix64_uniforms(s, 2)
        out.append(dict(model="anderson", L=L_lo + int(L_span * u0), t=1.0, W=W_lo + W_span * u1, seed=s,
                        skip=2))
    return out
