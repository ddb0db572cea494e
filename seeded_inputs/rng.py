"""Seeded random inputs shared by the oracle and the GPU path.

Nothing here is part of the integration method: this module only draws
the random numbers that the randomised lattice rule consumes (the m shift
vectors of the shifted rank-1 lattice rule, Section III, Eq. 18) and the
random kinematic points and arrival times of the batched and serving
workloads.  Both sides receive these numbers as plain inputs.

The generator is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): a 64-bit Weyl sequence
with increment 0x9E3779B97F4A7C15 followed by the published finaliser.
"""

from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, count: int) -> list[int]:
    """Return the first ``count`` outputs of SplitMix64 started at ``seed``."""
    state = seed & _MASK
    out = []
    for _ in range(count):
        state = (state + _GAMMA) & _MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        out.append(z ^ (z >> 31))
    return out


def uniform53(seed: int, count: int) -> np.ndarray:
    """``count`` doubles in [0, 1): the top 53 bits of each SplitMix64 output."""
    words = splitmix64(seed, count)
    return np.array([(w >> 11) * 2.0 ** -53 for w in words], dtype=np.float64)


def shift_table(seed: int, m: int, dmax: int) -> np.ndarray:
    """The m random shift vectors Delta_k in [0,1)^dmax (Section III, Eq. 18).

    Row k is shift k; component j is drawn k-major then j, so a sector of
    dimension d < dmax uses the first d components of every shift.
    """
    if m < 1 or dmax < 1:
        raise ValueError("need m >= 1 and dmax >= 1")
    return uniform53(seed, m * dmax).reshape(m, dmax)
