"""Deterministic search for the n = 882, k = 24 stand-in code.

The B1 code of Section IV is cited but its polynomials are not printed, so a
stand-in of the same length and dimension is drawn in the bivariate-bicycle form
over l = 63, m = 7 (A and B 441 x 441, H_X = [A | B], H_Z = [B^T | A^T]).

Rule: for draw d = 0, 1, 2, ... take ``numpy.random.Generator(PCG64(d))`` and
choose 3 distinct monomials x^a y^b (a < 63, b < 7, sampled without replacement
from the 441 exponent pairs in lexicographic order) for A, then 3 for B.  Accept
the first draw whose code has k = n - rank H_X - rank H_Z = 24, no 4-cycles
(no two rows of H_X, nor of H_Z, share two columns) and connected Tanner graphs.

Run as ``python -m workloads.search_qc882``; it prints the terms stored in
``codes.py``.  This is input generation: the rank routine below exists only to
choose the code and shares nothing with the decoder or the oracle.
"""

from __future__ import annotations

import sys

import numpy as np

from .codes import bb_code

L_ORDER, M_ORDER = 63, 7


def gf2_rank(h: np.ndarray) -> int:
    a = np.packbits(h.astype(np.uint8), axis=1, bitorder="little")
    a = a.copy()
    rows, ncols = a.shape[0], h.shape[1]
    r = 0
    for c in range(ncols):
        byte, bit = c >> 3, np.uint8(1 << (c & 7))
        col = (a[r:, byte] & bit) != 0
        hits = np.nonzero(col)[0]
        if hits.size == 0:
            continue
        p = r + hits[0]
        if p != r:
            a[[r, p]] = a[[p, r]]
        mask = (a[:, byte] & bit) != 0
        mask[r] = False
        a[mask] ^= a[r]
        r += 1
        if r == rows:
            break
    return r


def has_4cycle(h: np.ndarray) -> bool:
    g = h.astype(np.int32) @ h.T.astype(np.int32)
    np.fill_diagonal(g, 0)
    return bool((g >= 2).any())


def connected(h: np.ndarray) -> bool:
    m, n = h.shape
    seen_c = np.zeros(m, dtype=bool)
    seen_v = np.zeros(n, dtype=bool)
    frontier = [0]
    seen_c[0] = True
    while frontier:
        rows = np.array(frontier)
        vs = np.nonzero(h[rows].any(axis=0) & ~seen_v)[0]
        seen_v[vs] = True
        cs = np.nonzero(h[:, vs].any(axis=1) & ~seen_c)[0] if vs.size else np.array([], int)
        seen_c[cs] = True
        frontier = list(cs)
    return bool(seen_c.all() and seen_v[h.any(axis=0)].all())


def draw(d: int):
    rng = np.random.Generator(np.random.PCG64(d))
    pairs = [(a, b) for a in range(L_ORDER) for b in range(M_ORDER)]
    ia = rng.choice(len(pairs), size=3, replace=False)
    ib = rng.choice(len(pairs), size=3, replace=False)
    return [pairs[i] for i in sorted(ia)], [pairs[i] for i in sorted(ib)]


def search(max_draws: int = 200000, verbose: bool = True):
    for d in range(max_draws):
        at, bt = draw(d)
        code = bb_code("qc882", L_ORDER, M_ORDER, at, bt)
        rx = gf2_rank(code.hx)
        k = code.n - 2 * rx
        if k != 24:
            continue
        rz = gf2_rank(code.hz)
        if code.n - rx - rz != 24:
            continue
        if has_4cycle(code.hx) or has_4cycle(code.hz):
            if verbose:
                print(f"draw {d}: k=24 but has 4-cycles", flush=True)
            continue
        if not (connected(code.hx) and connected(code.hz)):
            if verbose:
                print(f"draw {d}: k=24 but disconnected", flush=True)
            continue
        return d, at, bt
    raise RuntimeError("no draw found")


if __name__ == "__main__":
    d, at, bt = search(int(sys.argv[1]) if len(sys.argv) > 1 else 200000)
    print(f"draw {d}: A terms {at}  B terms {bt}")
