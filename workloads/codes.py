"""CSS code definitions used as decoder inputs.

A CSS code is given by two binary parity-check matrices H_X and H_Z with
H_X H_Z^T = 0 (Section II-A).  X errors are decoded with H_Z, Z errors with H_X.

Bivariate bicycle (BB) codes: with S_l the l x l cyclic shift, x = S_l (x) I_m and
y = I_l (x) S_m; A and B are sums of monomials x^a y^b, and
H_X = [A | B], H_Z = [B^T | A^T].  The three BB codes below are the public
definitions of [[72,12,6]], [[144,12,12]] and [[288,12,18]] cited in Section IV.

The n = 882, k = 24 code is a stand-in for the B1 code of Section IV, whose
polynomials are cited but not printed in the paper: a weight-3 + weight-3 pair
in the same BB form over l = 63, m = 7, found by the deterministic search in
``search_qc882.py`` (first draw with k = 24, no 4-cycles and a connected Tanner
graph).  Its distance is unknown.

The small codes (Steane, distance-3 surface code, 3x3 toric code) have n <= 20
so that decoders can be checked against brute-force enumeration.
"""

from __future__ import annotations

import dataclasses
from typing import Iterable, Sequence, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class CSSCode:
    name: str
    hx: np.ndarray  # uint8 [mx, n]
    hz: np.ndarray  # uint8 [mz, n]

    @property
    def n(self) -> int:
        return int(self.hx.shape[1])


def _shift(l: int) -> np.ndarray:
    s = np.zeros((l, l), dtype=np.uint8)
    s[np.arange(l), (np.arange(l) + 1) % l] = 1
    return s


def _mono(l: int, m: int, a: int, b: int) -> np.ndarray:
    x = np.kron(_shift(l), np.eye(m, dtype=np.uint8))
    y = np.kron(np.eye(l, dtype=np.uint8), _shift(m))
    return (np.linalg.matrix_power(x.astype(np.int64), a)
            @ np.linalg.matrix_power(y.astype(np.int64), b)).astype(np.uint8) % 2


def bb_code(name: str, l: int, m: int,
            a_terms: Iterable[Tuple[int, int]],
            b_terms: Iterable[Tuple[int, int]]) -> CSSCode:
    """Bivariate bicycle code; each term (a, b) is the monomial x^a y^b."""
    lm = l * m
    A = np.zeros((lm, lm), dtype=np.uint8)
    B = np.zeros((lm, lm), dtype=np.uint8)
    for a, b in a_terms:
        A ^= _mono(l, m, a, b)
    for a, b in b_terms:
        B ^= _mono(l, m, a, b)
    hx = np.concatenate([A, B], axis=1)
    hz = np.concatenate([B.T, A.T], axis=1)
    return CSSCode(name, np.ascontiguousarray(hx), np.ascontiguousarray(hz))


# A = x^3 + y + y^2, B = y^3 + x + x^2
_A_GROSS = [(3, 0), (0, 1), (0, 2)]
_B_GROSS = [(0, 3), (1, 0), (2, 0)]


def bb72() -> CSSCode:
    """[[72,12,6]]: l = m = 6, A = x^3 + y + y^2, B = y^3 + x + x^2."""
    return bb_code("bb72", 6, 6, _A_GROSS, _B_GROSS)


def bb144() -> CSSCode:
    """[[144,12,12]]: l = 12, m = 6, A = x^3 + y + y^2, B = y^3 + x + x^2."""
    return bb_code("bb144", 12, 6, _A_GROSS, _B_GROSS)


def bb288() -> CSSCode:
    """[[288,12,18]]: l = m = 12, A = x^3 + y^2 + y^7, B = y^3 + x + x^2."""
    return bb_code("bb288", 12, 12, [(3, 0), (0, 2), (0, 7)], _B_GROSS)


# Result of search_qc882.py (draw 6 is the first accepted draw under its rule);
# stored so the search does not rerun at import time.  Terms are (a, b) for
# x^a y^b with x of order 63 and y of order 7.
QC882_A = [(27, 6), (32, 4), (33, 5)]
QC882_B = [(23, 1), (23, 4), (41, 2)]


def qc882() -> CSSCode:
    """n = 882, k = 24 stand-in: BB form over l = 63, m = 7 (weight 6 rows)."""
    return bb_code("qc882", 63, 7, QC882_A, QC882_B)


def steane7() -> CSSCode:
    """[[7,1,3]] Steane code: H_X = H_Z = the [7,4] Hamming check matrix
    (column i is the binary expansion of i + 1)."""
    h = np.array([[((i + 1) >> b) & 1 for i in range(7)] for b in range(3)],
                 dtype=np.uint8)
    return CSSCode("steane7", h.copy(), h.copy())


def _hgp(h1: np.ndarray, h2: np.ndarray, name: str) -> CSSCode:
    """Hypergraph product: H_X = [H1 (x) I | I (x) H2^T], H_Z = [I (x) H2 | H1^T (x) I]."""
    r1, n1 = h1.shape
    r2, n2 = h2.shape
    hx = np.concatenate([np.kron(h1, np.eye(n2, dtype=np.uint8)),
                         np.kron(np.eye(r1, dtype=np.uint8), h2.T)], axis=1) % 2
    hz = np.concatenate([np.kron(np.eye(n1, dtype=np.uint8), h2),
                         np.kron(h1.T, np.eye(r2, dtype=np.uint8))], axis=1) % 2
    return CSSCode(name, hx.astype(np.uint8), hz.astype(np.uint8))


def surface13() -> CSSCode:
    """Distance-3 planar surface code [[13,1,3]]: hypergraph product of the
    [3,1] repetition code's 2 x 3 check matrix with itself."""
    rep = np.array([[1, 1, 0], [0, 1, 1]], dtype=np.uint8)
    return _hgp(rep, rep, "surface13")


def toric18() -> CSSCode:
    """3 x 3 toric code [[18,2,3]]: hypergraph product of the cyclic 3 x 3
    repetition check matrix with itself."""
    rep = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 1]], dtype=np.uint8)
    return _hgp(rep, rep, "toric18")


def fig2_matrix() -> np.ndarray:
    """The 4 x 6 parity-check matrix of the worked example (Fig. 2)."""
    return np.array([[1, 1, 1, 0, 0, 0],
                     [0, 1, 1, 0, 0, 1],
                     [1, 0, 0, 1, 1, 0],
                     [0, 0, 0, 1, 1, 1]], dtype=np.uint8)


def to_csr(h: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Dense 0/1 matrix -> (row_ptr int32[m+1], col_idx int32[nnz]), columns ascending."""
    h = np.asarray(h, dtype=np.uint8)
    rows, cols = np.nonzero(h)
    row_ptr = np.zeros(h.shape[0] + 1, dtype=np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, cols.astype(np.int32)


def from_terms(terms: Sequence[Sequence[int]]):
    return [tuple(int(v) for v in t) for t in terms]
