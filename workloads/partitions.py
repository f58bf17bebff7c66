"""Representations of one partition of the checks, for the tree-vs-random
augmentation comparison of the paper's Table II (Section IV-A).

A partition is the list of maximal subtrees that Algorithm 2 finds for one root
order pi_k; it is an INPUT here (computed by the caller with the library's or
the oracle's Algorithm 2).  This module only packages it and draws the random
rows of the matched control, so it holds none of the decoder's arithmetic.

* tree: one representation [H; H_t] per subtree t, its rows in acceptance order;
* random: for each subtree, as many distinct rows of H drawn uniformly at random
  (numpy PCG64 seeded with (seed, 7919, k)), i.e. the same appended-row counts
  with the tree structure removed.

With ``count`` larger than the number of subtrees the list is cycled, so both
CSS parts can run the same number of representations.
"""

from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np


def _pack(row_lists: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    bp, rows = [0], []
    for r in row_lists:
        rows += [int(x) for x in r]
        bp.append(len(rows))
    return np.asarray(bp, np.int32), np.asarray(rows, np.int32)


def tree_bases(subtrees: Sequence[Sequence[int]], count: Optional[int] = None):
    """(basis_ptr, rows) with one representation per subtree (cycled to `count`)."""
    ns = len(subtrees)
    if ns == 0:
        raise ValueError("empty partition")
    k = ns if count is None else int(count)
    return _pack([subtrees[i % ns] for i in range(k)])


def matched_random_bases(subtrees: Sequence[Sequence[int]], m: int, seed: int, k: int,
                         count: Optional[int] = None):
    """(basis_ptr, rows): representation i appends len(subtrees[i % ns]) distinct rows
    of H (0 <= row < m) drawn at random."""
    ns = len(subtrees)
    if ns == 0:
        raise ValueError("empty partition")
    rng = np.random.Generator(np.random.PCG64([int(seed), 7919, int(k)]))
    out: List[List[int]] = []
    for i in range(ns if count is None else int(count)):
        size = len(subtrees[i % ns])
        out.append([int(x) for x in rng.choice(m, size, replace=False)])
    return _pack(out)
