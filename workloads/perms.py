"""Seeded permutations of the check nodes (the root order pi of Algorithm 2).

pi_0 is the identity; pi_k for k >= 1 is a uniform permutation drawn from
``numpy.random.Generator(PCG64([seed, k]))``.  Both the oracle and the library
take these arrays as inputs; neither draws permutations itself.
"""

from __future__ import annotations

import numpy as np


def check_permutations(m: int, count: int, seed: int = 0) -> np.ndarray:
    """int32 [count, m]; row 0 is the identity."""
    out = np.empty((count, m), dtype=np.int32)
    for k in range(count):
        if k == 0:
            out[k] = np.arange(m, dtype=np.int32)
        else:
            rng = np.random.Generator(np.random.PCG64([int(seed), k]))
            out[k] = rng.permutation(m).astype(np.int32)
    return out
