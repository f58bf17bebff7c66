"""Python driver for the plain CPU oracle of MBBP-LD.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The HIP library never imports,
links or calls anything here, and nothing here touches the HIP library.

The arithmetic lives in ``mbbp_oracle.c``; this module only marshals numpy
arrays.  Two builds exist: ``precision="f64"`` (REAL = double, the FP64 oracle)
and ``precision="f32"`` (REAL = float, every floating-point decision taken in
single precision in the same order as written in the C source).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbbp_oracle.c")
_LIBS: Dict[str, ctypes.CDLL] = {}

ORC_OK, ORC_EINVAL, ORC_ENOTINROWSPACE, ORC_ENOMEM = 0, -1, -2, -3

FLOODING, LAYERED = 0, 1
NMS, SPA, WNMS = 0, 1, 2
DEPOLARIZING, BSC_X = 0, 1  # noise models of sample()
MIN_WEIGHT, FWS = 0, 1


def lib_path(precision: str) -> str:
    return os.path.join(_HERE, f"liboracle_{precision}.so")


def build(force: bool = True) -> None:
    """Compile both oracle variants with gcc (no contraction, no fast math)."""
    for prec, extra in (("f64", []), ("f32", ["-DREAL=float", "-DORACLE_SINGLE"])):
        out = lib_path(prec)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
            continue
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", *extra, "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def _lib(precision: str = "f64") -> ctypes.CDLL:
    if precision not in ("f64", "f32"):
        raise ValueError(precision)
    if precision not in _LIBS:
        path = lib_path(precision)
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ctypes.CDLL(path)
        _declare(lib)
        _LIBS[precision] = lib
    return _LIBS[precision]


_P = ctypes.c_void_p


def _declare(lib: ctypes.CDLL) -> None:
    i32, i64, u64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.orc_philox4x64_10.argtypes = [_P, _P, _P]
    lib.orc_philox4x64_10.restype = None
    lib.orc_sample.argtypes = [i32, i32, _P, _P, i32, _P, _P, u64, dbl, i32, i64, i64, _P, _P, _P, _P]
    lib.orc_rank.argtypes = [i32, i32, _P, _P]
    lib.orc_subtrees.argtypes = [i32, i32, _P, _P, _P, _P, _P, _P]
    lib.orc_build_bases.argtypes = [i32, i32, _P, _P, i32, i32, i32, _P, _P, _P, i32]
    lib.orc_decode.argtypes = [i32, i32, _P, _P, i32, _P, _P, _P, i32, i32, i32, dbl, dbl, i32,
                               i64, _P, i32, _P, _P, _P, _P, _P, _P, _P, i32, _P, _P, _P, _P]
    lib.orc_failures.argtypes = [i32, i32, _P, _P, i64, _P, _P, _P]
    lib.orc_in_rowspace.argtypes = [i32, i32, _P, _P, i32, _P, _P, _P]
    lib.orc_real_bytes.argtypes = []
    lib.orc_select.argtypes = [i32, i32, i64, _P, _P, i32, _P]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(status: int, what: str) -> None:
    if status != ORC_OK:
        names = {ORC_EINVAL: "EINVAL", ORC_ENOTINROWSPACE: "ENOTINROWSPACE", ORC_ENOMEM: "ENOMEM"}
        raise OracleError(status, f"{what}: {names.get(status, status)}")


class OracleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


def csr(h: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    h = np.asarray(h, dtype=np.uint8)
    rows, cols = np.nonzero(h)
    ptr = np.zeros(h.shape[0] + 1, dtype=np.int32)
    np.add.at(ptr, rows + 1, 1)
    return np.cumsum(ptr).astype(np.int32), np.ascontiguousarray(cols, dtype=np.int32)


def words64(bits: int) -> int:
    return (bits + 63) // 64


# ---------------------------------------------------------------------------- noise

def philox4x64_10(ctr: Sequence[int], key: Sequence[int], precision: str = "f64") -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    _lib(precision).orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sample(hx: np.ndarray, hz: np.ndarray, seed: int, p: float, shot0: int, shots: int,
           noise: int = DEPOLARIZING):
    """Errors and syndromes for shots [shot0, shot0 + shots): depolarizing (X, Y, Z
    each with probability p/3), or BSC_X (X errors only, each qubit flipped with
    probability p: the noise of the paper's experiments, Section IV).
    Returns (e_x, e_z, s_x, s_z) as bit-packed uint64 arrays, named by error
    type: s_x = H_Z e_x (m_Z bits), s_z = H_X e_z (m_X bits)."""
    lib = _lib("f64")
    n = hx.shape[1]
    xp, xi = csr(hx)
    zp, zi = csr(hz)
    wn, wx, wz = words64(n), words64(hx.shape[0]), words64(hz.shape[0])
    ex = np.zeros((shots, wn), np.uint64)
    ez = np.zeros((shots, wn), np.uint64)
    sx = np.zeros((shots, wz), np.uint64)
    sz = np.zeros((shots, wx), np.uint64)
    _check(lib.orc_sample(n, hx.shape[0], _ptr(xp), _ptr(xi), hz.shape[0], _ptr(zp), _ptr(zi),
                          int(seed), float(p), int(noise), int(shot0), int(shots),
                          _ptr(ex), _ptr(ez), _ptr(sx), _ptr(sz)), "sample")
    return ex, ez, sx, sz


# ---------------------------------------------------------------------------- GF(2)

def rank(h: np.ndarray) -> int:
    ptr, idx = csr(h)
    r = _lib("f64").orc_rank(h.shape[0], h.shape[1], _ptr(ptr), _ptr(idx))
    if r < 0:
        _check(r, "rank")
    return int(r)


def in_rowspace(h: np.ndarray, rows: np.ndarray) -> np.ndarray:
    ptr, idx = csr(h)
    qp, qi = csr(np.atleast_2d(rows))
    out = np.zeros(qp.shape[0] - 1, np.uint8)
    _check(_lib("f64").orc_in_rowspace(h.shape[0], h.shape[1], _ptr(ptr), _ptr(idx), out.shape[0],
                                       _ptr(qp), _ptr(qi), _ptr(out)), "in_rowspace")
    return out.astype(bool)


# ---------------------------------------------------------------------------- Algorithm 2

def subtrees(h: np.ndarray, perm: Sequence[int]):
    """Algorithm 2.  Returns (check_sets int32[m] 1-based, order int32[m], n_subtrees)."""
    ptr, idx = csr(h)
    m = h.shape[0]
    pm = np.ascontiguousarray(perm, dtype=np.int32)
    cs = np.zeros(m, np.int32)
    order = np.zeros(m, np.int32)
    ns = np.zeros(1, np.int32)
    _check(_lib("f64").orc_subtrees(m, h.shape[1], _ptr(ptr), _ptr(idx), _ptr(pm), _ptr(cs),
                                    _ptr(order), _ptr(ns)), "subtrees")
    return cs, order, int(ns[0])


def subtree_lists(h: np.ndarray, perm: Sequence[int]):
    """The subtrees of Algorithm 2 as row lists in acceptance order."""
    cs, order, ns = subtrees(h, perm)
    return [[int(c) for c in order if cs[c] == s] for s in range(1, ns + 1)]


BASIS_MODES = {"subtrees": 0, "ramp": 1}


def build_bases(h: np.ndarray, mode: str, L: int, perms: np.ndarray):
    """Returns (basis_ptr int32[L+1], rows int32[]) of duplicated H rows."""
    ptr, idx = csr(h)
    m = h.shape[0]
    pm = np.ascontiguousarray(perms, dtype=np.int32)
    cap = L * m
    bp = np.zeros(L + 1, np.int32)
    rows = np.zeros(max(cap, 1), np.int32)
    _check(_lib("f64").orc_build_bases(m, h.shape[1], _ptr(ptr), _ptr(idx), BASIS_MODES[mode], L,
                                       pm.shape[0], _ptr(pm), _ptr(bp), _ptr(rows), cap),
           "build_bases")
    return bp, rows[: bp[-1]].copy()


# ---------------------------------------------------------------------------- decoding

@dataclass
class DecodeResult:
    cand: np.ndarray      # uint64 [shots, L, words]
    K: np.ndarray         # int32 [shots, L]
    conv: np.ndarray      # bool [shots, L]
    llr: Optional[np.ndarray]
    margin: np.ndarray    # float64 [shots, L, 2]: min |q| at signs, min |P| at decisions
    clamp: np.ndarray     # bool [shots, L]
    chosen: np.ndarray    # int32 [shots]
    corr: np.ndarray      # uint64 [shots, words]


def appended_rows(h: np.ndarray, basis_ptr: np.ndarray, rows: np.ndarray,
                  explicit: Optional[Dict[int, np.ndarray]] = None):
    """Appended rows as explicit CSR: row indices >= 0 duplicate H rows; a
    negative index -k-1 takes ``explicit[k]`` (a 0/1 row)."""
    dense = []
    for r in rows:
        r = int(r)
        dense.append(h[r] if r >= 0 else np.asarray(explicit[-r - 1], np.uint8))
    if not dense:
        return np.zeros(1, np.int32), np.zeros(0, np.int32)
    return csr(np.array(dense, dtype=np.uint8))


def decode(h: np.ndarray, basis_ptr: np.ndarray, rows: np.ndarray, syn: np.ndarray,
           prior: np.ndarray, T: int, schedule: int = FLOODING, rule: int = NMS,
           alpha: float = 0.875, rmax: float = 65536.0, fixed_T: bool = False,
           select_rule: int = MIN_WEIGHT, want_llr: bool = False, precision: str = "f64",
           explicit: Optional[Dict[int, np.ndarray]] = None,
           walpha: Optional[np.ndarray] = None, wbeta: Optional[np.ndarray] = None) -> DecodeResult:
    """BP on every representation and the list decision (Algorithm 1).  rule WNMS
    is the weighted min-sum with damping; walpha, wbeta are [T][L] (iteration t at
    row t - 1) and margin[..., 0] is then the distance to the nearest non-smooth
    point of the forward map."""
    lib = _lib(precision)
    m, n = h.shape
    ptr, idx = csr(h)
    bp = np.ascontiguousarray(basis_ptr, np.int32)
    L = bp.shape[0] - 1
    ap, ai = appended_rows(h, bp, rows, explicit)
    syn = np.ascontiguousarray(syn, np.uint64)
    shots = syn.shape[0]
    prior = np.ascontiguousarray(prior, np.float64)
    per_shot = 1 if prior.ndim == 2 else 0
    wn = words64(n)
    cand = np.zeros((shots, L, wn), np.uint64)
    K = np.zeros((shots, L), np.int32)
    conv = np.zeros((shots, L), np.uint8)
    llr = np.zeros((shots, L, n), np.float64) if want_llr else None
    margin = np.zeros((shots, L, 2), np.float64)
    clamp = np.zeros((shots, L), np.uint8)
    chosen = np.zeros(shots, np.int32)
    corr = np.zeros((shots, wn), np.uint64)
    wa = wb = None
    if rule == WNMS:
        wa = np.ascontiguousarray(walpha, np.float64).reshape(int(T), L)
        wb = np.ascontiguousarray(wbeta, np.float64).reshape(int(T), L)
    _check(lib.orc_decode(m, n, _ptr(ptr), _ptr(idx), L, _ptr(bp), _ptr(ap), _ptr(ai),
                          int(T), int(schedule), int(rule), float(alpha), float(rmax),
                          1 if fixed_T else 0, shots, _ptr(prior), per_shot, _ptr(syn),
                          _ptr(cand), _ptr(K), _ptr(conv), _ptr(llr), _ptr(margin), _ptr(clamp),
                          int(select_rule), _ptr(chosen), _ptr(corr), _ptr(wa), _ptr(wb)), "decode")
    return DecodeResult(cand, K, conv.astype(bool), llr, margin, clamp.astype(bool), chosen, corr)


def select(cand: np.ndarray, conv: np.ndarray, rule: int = MIN_WEIGHT) -> np.ndarray:
    """Decision rule on given lists: cand uint64 [shots, L, W], conv bool [shots, L]."""
    cand = np.ascontiguousarray(cand, np.uint64)
    cv = np.ascontiguousarray(conv, np.uint8)
    out = np.zeros(cand.shape[0], np.int32)
    _check(_lib("f64").orc_select(cand.shape[1], cand.shape[2], cand.shape[0], _ptr(cand), _ptr(cv),
                                  int(rule), _ptr(out)), "select")
    return out


def failures(stab: np.ndarray, err: np.ndarray, corr: np.ndarray) -> np.ndarray:
    """fail[s] = residual err ^ corr is not in the row space of ``stab``."""
    ptr, idx = csr(stab)
    err = np.ascontiguousarray(err, np.uint64)
    corr = np.ascontiguousarray(corr, np.uint64)
    out = np.zeros(err.shape[0], np.uint8)
    _check(_lib("f64").orc_failures(stab.shape[0], stab.shape[1], _ptr(ptr), _ptr(idx),
                                    err.shape[0], _ptr(err), _ptr(corr), _ptr(out)), "failures")
    return out.astype(bool)


def prior_llr(p: float, noise: int = DEPOLARIZING) -> float:
    """Per-type prior LLR (BP initialisation of Section II-B): ln((1 - q) / q) with
    q = 2p/3 under depolarizing noise (each of the X and Z parts flips with that
    probability) and q = p under X-only noise (the binary symmetric channel)."""
    q = p if noise == BSC_X else 2.0 * p / 3.0
    return float(np.log((1.0 - q) / q))


def unpack(words: np.ndarray, n: int) -> np.ndarray:
    """uint64 [..., W] LSB-first -> uint8 [..., n]."""
    w = np.ascontiguousarray(words, dtype="<u8")
    b = np.unpackbits(w.view(np.uint8), axis=-1, bitorder="little")
    return b[..., :n]


def pack(bits: np.ndarray) -> np.ndarray:
    """uint8 [..., n] -> uint64 [..., ceil(n/64)] LSB-first."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = bits.shape[-1]
    pad = words64(n) * 64 - n
    if pad:
        bits = np.concatenate([bits, np.zeros(bits.shape[:-1] + (pad,), np.uint8)], axis=-1)
    by = np.packbits(bits, axis=-1, bitorder="little")
    return np.ascontiguousarray(by).view("<u8").astype(np.uint64)


@dataclass
class RunResult:
    fails: int
    shots: int
    sum_kmax: int
    sum_k: int
    edge_updates: int


def run(code, bases_x, bases_z, seed: int, p: float, shot0: int, shots: int, T: int,
        alpha: float, schedule: int = FLOODING, rule: int = NMS, select_rule: int = MIN_WEIGHT,
        rmax: float = 65536.0, precision: str = "f64", noise: int = DEPOLARIZING) -> RunResult:
    """The whole path on the CPU for a shot range: sample, decode both types,
    select, failure test, counters.  bases_* = (basis_ptr, rows).  Both parts
    take the prior of the noise model (under X-only noise part Z sees no errors)."""
    ex, ez, sx, sz = sample(code.hx, code.hz, seed, p, shot0, shots, noise)
    mu = prior_llr(p, noise)
    mu32 = float(np.float32(mu))
    n = code.n
    fails = np.zeros(shots, bool)
    kmax = np.zeros(shots, np.int64)
    sum_k = 0
    edges = 0
    # part X: e_x, s_x = H_Z e_x, representations of H_Z (bases_z), stabilizers H_X;
    # part Z: e_z, s_z = H_X e_z, representations of H_X (bases_x), stabilizers H_Z.
    for h, (bp, rows), syn, err, stab in ((code.hz, bases_z, sx, ex, code.hx),
                                           (code.hx, bases_x, sz, ez, code.hz)):
        res = decode(h, bp, rows, syn, np.full(n, mu32), T, schedule, rule, alpha, rmax,
                     select_rule=select_rule, precision=precision)
        fails |= failures(stab, err, res.corr)
        kmax = np.maximum(kmax, res.K.max(axis=1))
        sum_k += int(res.K.sum())
        E = h.sum() + np.array([h[rows[bp[l]:bp[l + 1]]].sum() for l in range(len(bp) - 1)])
        edges += int((res.K * E[None, :]).sum())
    return RunResult(int(fails.sum()), shots, int(kmax.sum()), sum_k, edges)
