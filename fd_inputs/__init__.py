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
