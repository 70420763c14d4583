"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no hierarchization arithmetic: it only describes grids
(level vectors, shapes, combination-technique sets) and draws seeded values.
Both the GPU path and the CPU oracle take their inputs from here.

Grid convention: a level vector ``(l_0, ..., l_{d-1})`` (level 1 = one point,
so axis k has ``2**l_k - 1`` interior points, zero boundary not stored); the
array shape is the reversed tuple of point counts, so grid axis 0 is the last
(contiguous) array axis.
"""
from __future__ import annotations

from math import comb
from typing import List, Sequence, Tuple

import numpy as np

# Workloads (sizes as in the paper's experiments: double precision grids of up
# to about 1 GB, |l|_1 = 27 <-> 1 GB; d = 2..5 grids of 125-500 MB, Section 4).
SMALL_2D = (5, 5)                 # 31 x 31 points
ANISO_3D = (10, 9, 8)             # 1023 x 511 x 255 = 133,302,015 points, 1.07 GB FP64
ANISO_5D = (6, 6, 5, 5, 5)        # 63 x 63 x 31 x 31 x 31 = 118,240,479 points, 0.95 GB FP64
COMBI_D, COMBI_N = 4, 10          # combination set: 589 grids, 980,797 points


def points_per_axis(levels: Sequence[int]) -> List[int]:
    return [(1 << int(l)) - 1 for l in levels]


def shape_of(levels: Sequence[int]) -> Tuple[int, ...]:
    """Array shape of a grid: reversed point counts (axis 0 last, contiguous)."""
    return tuple(reversed(points_per_axis(levels)))


def num_points(levels: Sequence[int]) -> int:
    n = 1
    for c in points_per_axis(levels):
        n *= c
    return n


def _compositions(total: int, parts: int, minimum: int = 1):
    """All tuples of `parts` integers >= minimum summing to `total`, lexicographic."""
    if parts == 1:
        if total >= minimum:
            yield (total,)
        return
    for first in range(minimum, total - minimum * (parts - 1) + 1):
        for rest in _compositions(total - first, parts - 1, minimum):
            yield (first,) + rest


def combination_set(d: int = COMBI_D, n: int = COMBI_N):
    """Level vectors and coefficients of the classical combination technique.

    All level vectors with every l_k >= 1 and |l|_1 = n + d - 1 - q for
    q = 0..d-1, weighted by (-1)^q * binom(d-1, q) (in two dimensions the
    weights are +1 and -1, as in Fig. 1).  Order: q ascending, then
    lexicographic.  Returns (levels_list, coefficients_list)."""
    levels, coefs = [], []
    for q in range(d):
        c = (-1) ** q * comb(d - 1, q)
        for lv in _compositions(n + d - 1 - q, d, 1):
            levels.append(lv)
            coefs.append(c)
    return levels, coefs


def uniform(levels: Sequence[int], seed, dtype=np.float64) -> np.ndarray:
    """i.i.d. uniform[-1, 1] values drawn in float64 from default_rng(seed), cast to dtype."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=shape_of(levels))
    return x.astype(dtype, copy=False)


def coordinates(level: int) -> np.ndarray:
    """Interior grid coordinates i / 2^l, i = 1 .. 2^l - 1, of one axis."""
    return np.arange(1, 1 << level, dtype=np.float64) / float(1 << level)


def sine_plus_noise(levels: Sequence[int], seed, noise: float = 0.01, dtype=np.float64) -> np.ndarray:
    """f(x) = prod_k sin(pi x_k) + noise * N(0, 1), noise drawn from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    shape = shape_of(levels)
    out = np.ones(shape, dtype=np.float64)
    d = len(levels)
    for k, l in enumerate(levels):
        s = np.sin(np.pi * coordinates(l))
        view = [1] * d
        view[d - 1 - k] = s.size
        out *= s.reshape(view)
    out += noise * rng.standard_normal(size=shape)
    return out.astype(dtype, copy=False)


def combination_values(levels_list, seed: int = 3, dtype=np.float64) -> List[np.ndarray]:
    """Values of a combination set: grid g gets uniform[-1,1] from default_rng([seed, g])."""
    return [uniform(lv, [seed, g], dtype) for g, lv in enumerate(levels_list)]


def fd_entries(levels_list, count: int = 64, seed: int = 4):
    """`count` random (grid, flat index) pairs for finite-difference checks."""
    rng = np.random.default_rng(seed)
    sizes = np.array([num_points(lv) for lv in levels_list])
    grids = rng.integers(0, len(levels_list), size=count)
    flat = np.array([rng.integers(0, sizes[g]) for g in grids])
    return list(zip(grids.tolist(), flat.tolist()))
