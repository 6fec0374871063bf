"""FP64 oracle of the ACUI point grid (TEST INFRASTRUCTURE ONLY).

Sec. 3.3, Eq. 13: a cuboid of size S1 x S2 x S3 centred on the world
origin is divided into an M1 x M2 x M3 voxel grid, and Gaussian centres are
placed at (n1 S1 d / M1, n2 S2 d / M2, n3 S3 d / M3) for every integer
triple with |n_i| <= [M_i / (2 d)] + 1.

Readings: [.] is the integer part (floor, M_i / (2 d) is positive).  Each
coordinate is evaluated in float64 as ((n_i * S_i) * d) / M_i and rounded
once to float32.  Points are listed with n1 slowest and n3 fastest, each
n_i ascending (C order of the index grid); the paper fixes no order.
"""
from __future__ import annotations

import math

import numpy as np


def half_extent(m: int, d: float) -> int:
    """K_i = [M_i / (2 d)] + 1: n_i runs over -K_i .. K_i."""
    return int(math.floor(m / (2.0 * d))) + 1


def count(size, grid, d: float) -> int:
    """Number of ACUI points, prod_i (2 K_i + 1)."""
    return int(np.prod([2 * half_extent(m, d) + 1 for m in grid]))


def points(size, grid, d: float) -> np.ndarray:
    """The ACUI centres, float32 [count, 3] (Eq. 13)."""
    axes = []
    for s, m in zip(size, grid):
        k = half_extent(m, d)
        n = np.arange(-k, k + 1, dtype=np.float64)
        axes.append(((n * float(s)) * float(d)) / float(m))
    a1, a2, a3 = np.meshgrid(*axes, indexing="ij")
    p = np.stack([a1.reshape(-1), a2.reshape(-1), a3.reshape(-1)], axis=1)
    return np.ascontiguousarray(p.astype(np.float32))
