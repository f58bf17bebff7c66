"""Pins of the CPU oracle against facts the paper and mathematics fix.

None of these retypes the oracle's own formulas: each compares against a worked
example printed in the paper, a library routine, a closed form, an invariant,
or brute-force enumeration on tiny inputs.
"""

import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from workloads import codes
from workloads.perms import check_permutations

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ Philox (noise)

def _numpy_philox_block(ctr, key):
    """numpy's Philox advances its 256-bit counter before producing a block, so
    the block for counter c is the first output of a generator started at c - 1."""
    c = [int(x) for x in ctr]
    total = c[0] | (c[1] << 64) | (c[2] << 128) | (c[3] << 192)
    total = (total - 1) % (1 << 256)
    start = [(total >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(start, dtype=np.uint64),
                          key=np.array([int(k) for k in key], dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([1, 0, 0, 0], [0, 0]),
    ([12345, 17, 0, 0], [1, 0]),
    ([2**64 - 1, 5, 3, 1], [0xDEADBEEF, 42]),
    ([7, 2**63, 0, 2**64 - 1], [2**64 - 1, 2**64 - 1]),
])
def test_philox_matches_numpy(ctr, key):
    np.testing.assert_array_equal(oracle.philox4x64_10(ctr, key), _numpy_philox_block(ctr, key))


@pytest.mark.parametrize("p", [0.01, 0.02, 0.03, 0.04, 0.05, 0.06, 0.08, 0.1, 0.5])
def test_thresholds_equal_exact_floor(p):
    """The double-precision thresholds floor(k p/3 2^32) equal the exact rational
    floor for the error rates used (so no rounding ambiguity exists there)."""
    for k in (1, 2, 3):
        exact = (Fraction(k) * Fraction(p) / 3 * 2**32).__floor__()
        approx = int(np.floor(k * (p / 3.0) * 4294967296.0))
        assert exact == approx


def test_sampler_against_numpy_philox_and_matmul():
    """Errors re-derived from numpy's Philox stream with exact rational thresholds,
    syndromes from an integer matrix product."""
    code = codes.bb72()
    seed, p, shot0, shots = 1, 0.05, 1000, 40
    ex, ez, sx, sz = oracle.sample(code.hx, code.hz, seed, p, shot0, shots)
    n = code.n
    t = [(Fraction(k) * Fraction(p) / 3 * 2**32).__floor__() for k in (1, 2, 3)]
    bx = np.zeros((shots, n), np.uint8)
    bz = np.zeros((shots, n), np.uint8)
    for s in range(shots):
        for b in range((n + 7) // 8):
            out = _numpy_philox_block([shot0 + s, b, 0, 0], [seed, 0])
            for sub in range(8):
                q = 8 * b + sub
                if q >= n:
                    break
                u = (int(out[sub // 2]) >> (32 * (sub % 2))) & 0xFFFFFFFF
                if u < t[0]:
                    bx[s, q] = 1
                elif u < t[1]:
                    bx[s, q] = bz[s, q] = 1
                elif u < t[2]:
                    bz[s, q] = 1
    np.testing.assert_array_equal(oracle.unpack(ex, n), bx)
    np.testing.assert_array_equal(oracle.unpack(ez, n), bz)
    np.testing.assert_array_equal(oracle.unpack(sx, code.hz.shape[0]),
                                  (bx.astype(np.int64) @ code.hz.T.astype(np.int64)) % 2)
    np.testing.assert_array_equal(oracle.unpack(sz, code.hx.shape[0]),
                                  (bz.astype(np.int64) @ code.hx.T.astype(np.int64)) % 2)


def test_sampler_frequencies():
    """X-only, Y and Z-only frequencies each p/3 within 5 binomial sigmas."""
    code = codes.bb144()
    p, shots = 0.06, 20000
    ex, ez, _, _ = oracle.sample(code.hx, code.hz, 7, p, 0, shots)
    bx = oracle.unpack(ex, code.n).astype(bool)
    bz = oracle.unpack(ez, code.n).astype(bool)
    N = bx.size
    for cnt in ((bx & ~bz).sum(), (bx & bz).sum(), (~bx & bz).sum()):
        mean = N * p / 3
        assert abs(cnt - mean) < 5 * np.sqrt(mean * (1 - p / 3))


def test_sampler_x_only_against_numpy_philox():
    """X-only noise (the binary symmetric channel of Section IV): qubit q flipped iff
    its Philox word u < floor(p 2^32) (exact rational floor), no Z errors, s_z = 0."""
    code = codes.bb144()
    seed, p, shot0, shots = 3, 0.07, 55, 30
    ex, ez, sx, sz = oracle.sample(code.hx, code.hz, seed, p, shot0, shots, noise=oracle.BSC_X)
    n = code.n
    tb = (Fraction(p) * 2**32).__floor__()
    bx = np.zeros((shots, n), np.uint8)
    for s in range(shots):
        for b in range((n + 7) // 8):
            out = _numpy_philox_block([shot0 + s, b, 0, 0], [seed, 0])
            for sub in range(8):
                q = 8 * b + sub
                if q < n:
                    bx[s, q] = ((int(out[sub // 2]) >> (32 * (sub % 2))) & 0xFFFFFFFF) < tb
    np.testing.assert_array_equal(oracle.unpack(ex, n), bx)
    assert not ez.any() and not sz.any()
    np.testing.assert_array_equal(oracle.unpack(sx, code.hz.shape[0]),
                                  (bx.astype(np.int64) @ code.hz.T.astype(np.int64)) % 2)


def test_sampler_x_only_is_the_depolarizing_x_part():
    """With p_x = 2 p / 3 exact (p = 0.75: both thresholds are 2^31) the X-only
    errors are exactly the X parts (X or Y) of the depolarizing errors."""
    code = codes.bb72()
    dep = oracle.sample(code.hx, code.hz, 9, 0.75, 100, 50)
    bsc = oracle.sample(code.hx, code.hz, 9, 0.5, 100, 50, noise=oracle.BSC_X)
    np.testing.assert_array_equal(bsc[0], dep[0])
    np.testing.assert_array_equal(bsc[2], dep[2])


def test_sampler_x_only_frequency_and_prior():
    code = codes.bb144()
    p, shots = 0.04, 20000
    ex, _, _, _ = oracle.sample(code.hx, code.hz, 11, p, 0, shots, noise=oracle.BSC_X)
    cnt = int(oracle.unpack(ex, code.n).sum())
    mean = code.n * shots * p
    assert abs(cnt - mean) < 5 * np.sqrt(mean * (1 - p))
    # prior LLR of the binary symmetric channel, log((1 - p) / p), against the
    # depolarizing one at the rate with the same flip probability (2 p'/3 = p)
    assert oracle.prior_llr(p, oracle.BSC_X) == pytest.approx(np.log(0.96 / 0.04), rel=1e-15)
    assert oracle.prior_llr(p, oracle.BSC_X) == pytest.approx(oracle.prior_llr(1.5 * p), rel=1e-12)


# ------------------------------------------------------------------ codes and GF(2)

@pytest.mark.parametrize("factory,k", [(codes.bb72, 12), (codes.bb144, 12), (codes.bb288, 12),
                                       (codes.qc882, 24), (codes.steane7, 1),
                                       (codes.surface13, 1), (codes.toric18, 2)])
def test_code_dimension(factory, k):
    """k = n - rank H_X - rank H_Z equals the published [[n, k]] (Section IV)."""
    c = factory()
    assert not ((c.hx.astype(np.int64) @ c.hz.T.astype(np.int64)) % 2).any()
    assert c.n - oracle.rank(c.hx) - oracle.rank(c.hz) == k


def _span(h):
    """All vectors of the row space by enumeration (tiny h only)."""
    rows = [r.astype(np.uint8) for r in h]
    out = set()
    for coeffs in itertools.product([0, 1], repeat=len(rows)):
        v = np.zeros(h.shape[1], np.uint8)
        for c, r in zip(coeffs, rows):
            if c:
                v ^= r
        out.add(v.tobytes())
    return out


def test_rank_and_rowspace_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(30):
        m, n = rng.integers(1, 7), rng.integers(2, 10)
        h = (rng.random((m, n)) < 0.4).astype(np.uint8)
        span = _span(h)
        assert oracle.rank(h) == int(np.log2(len(span)))
        q = (rng.random((12, n)) < 0.5).astype(np.uint8)
        mem = oracle.in_rowspace(h, q)
        for row, got in zip(q, mem):
            assert got == (row.tobytes() in span)


# ------------------------------------------------------------------ Algorithm 2

def _read_fig2():
    rec = {}
    with open(os.path.join(GOLDEN, "fig2_subtrees.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            rec.setdefault(tok[0], []).append(tok[1:])
    h = np.array([[int(ch) for ch in row] for row in rec["H"][0]], np.uint8)
    perm = [int(x) for x in rec["perm"][0]]
    cs = [int(x) for x in rec["check_sets"][0]]
    subs = {int(t[0]): [int(x) for x in t[1:]] for t in rec["subtree"]}
    return h, perm, cs, subs


def test_fig2_worked_example():
    h, perm, cs_expect, subs = _read_fig2()
    np.testing.assert_array_equal(h, codes.fig2_matrix())
    cs, order, ns = oracle.subtrees(h, perm)
    assert list(cs) == cs_expect
    assert ns == len(subs)
    lists = oracle.subtree_lists(h, perm)
    for s, rows in subs.items():
        assert lists[s - 1] == rows


def _check_subtree_invariants(h, perm):
    m, n = h.shape
    cs, order, ns = oracle.subtrees(h, perm)
    assert sorted(order.tolist()) == list(range(m))           # every check once
    assert set(cs.tolist()) == set(range(1, ns + 1))           # a partition
    w = int(h.sum(axis=1).max())
    lists = oracle.subtree_lists(h, perm)
    for s, rows in enumerate(lists, start=1):
        sub = h[rows]
        covered = np.nonzero(sub.any(axis=0))[0]
        # acyclic and connected: a tree has #vars = sum(deg) - (#checks - 1)
        assert covered.size == int(sub.sum()) - (len(rows) - 1)
        # every prefix of the acceptance order is connected (BFS growth)
        seen = set(np.nonzero(h[rows[0]])[0])
        for r in rows[1:]:
            vs = set(np.nonzero(h[r])[0])
            assert len(vs & seen) == 1
            seen |= vs
        # maximality: a check unassigned while s was built (assigned later) that
        # touches s's variables touches at least two of them
        cov = set(covered.tolist())
        for c in range(m):
            if cs[c] > s:
                inter = len(set(np.nonzero(h[c])[0]) & cov)
                assert inter == 0 or inter >= 2
        # Lemma 1: |t| <= (|V_v| - 1) / (w - 1)
        assert len(rows) <= (n - 1) / (w - 1)
    # the root of each subtree is the first unassigned check in pi order
    roots = [rows[0] for rows in lists]
    pos = {c: i for i, c in enumerate(perm)}
    assert roots == sorted(roots, key=lambda c: pos[c])


@pytest.mark.parametrize("factory", [codes.bb72, codes.bb144, codes.bb288, codes.qc882])
def test_subtree_invariants(factory):
    c = factory()
    for h in (c.hx, c.hz):
        perms = check_permutations(h.shape[0], 3, seed=11)
        for perm in perms:
            _check_subtree_invariants(h, perm)


def test_bases_subtree_mode_and_ramp():
    c = codes.bb144()
    perms = check_permutations(72, 8, seed=0)
    bp, rows = oracle.build_bases(c.hx, "subtrees", 16, perms)
    sets = [frozenset(rows[bp[l]:bp[l + 1]].tolist()) for l in range(16)]
    assert len(set(sets)) == 16                                # distinct row sets
    all_subtrees = [frozenset(r) for k in range(8) for r in oracle.subtree_lists(c.hx, perms[k])]
    assert all(s in all_subtrees for s in sets)               # each is a maximal subtree
    c3 = codes.bb288()
    perms3 = check_permutations(144, 32, seed=0)
    bp3, rows3 = oracle.build_bases(c3.hx, "ramp", 32, perms3)
    sizes = np.diff(bp3)
    assert sizes[0] == 0 and sizes[-1] == 144
    assert all(sizes[l] == round(l * 144 / 31) for l in range(32))
    assert sorted(rows3[bp3[-2]:bp3[-1]].tolist()) == list(range(144))


# ------------------------------------------------------------------ BP closed forms

def _one_basis(h, rows):
    return np.array([0, len(rows)], np.int32), np.array(rows, np.int32)


@pytest.mark.parametrize("schedule", [oracle.FLOODING])
@pytest.mark.parametrize("mu,alpha,rmax", [(2.5, 0.75, 65536.0), (3.0, 0.875, 1.0)])
def test_iteration_one_closed_form(schedule, mu, alpha, rmax):
    """After one flooding iteration from uniform mu > 0 every check message is
    (-1)^{s_j} * min(alpha * mu, rmax), so P_i = mu + that summed over N(i)."""
    c = codes.bb72()
    h = c.hz
    bp, rows = _one_basis(h, [0, 5, 7])
    rng = np.random.default_rng(0)
    sb = (rng.random((6, h.shape[0])) < 0.3).astype(np.uint8)
    syn = oracle.pack(sb)
    res = oracle.decode(h, bp, rows, syn, np.full(h.shape[1], mu), T=1, schedule=schedule,
                        alpha=alpha, rmax=rmax, fixed_T=True, want_llr=True)
    haug = np.concatenate([h, h[rows]], axis=0).astype(np.int64)
    saug = np.concatenate([sb, sb[:, rows]], axis=1).astype(np.int64)
    mag = min(alpha * mu, rmax)
    expect = mu + mag * ((1 - 2 * saug) @ haug)
    np.testing.assert_allclose(res.llr[:, 0, :], expect, rtol=0, atol=1e-12)


def test_hand_example_schedules():
    """Two weight-2 checks sharing variable 1, s = (1, 0), mu = (2, 3, 4), alpha 1/2.
    By hand, one iteration gives
      flooding: r00 = -1.5, r01 = -1, r11 = 2, r12 = 1.5  -> P = (0.5, 4, 5.5)
      serial:   r00 = -1.5, r01 = -1, then q11 = 3 - 1 = 2: r11 = 2, r12 = 1 -> P = (0.5, 4, 5)."""
    h = np.array([[1, 1, 0], [0, 1, 1]], np.uint8)
    syn = oracle.pack(np.array([[1, 0]], np.uint8))
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    mu = np.array([2.0, 3.0, 4.0])
    fl = oracle.decode(h, bp, rows, syn, mu, T=1, schedule=oracle.FLOODING, alpha=0.5,
                       fixed_T=True, want_llr=True)
    se = oracle.decode(h, bp, rows, syn, mu, T=1, schedule=oracle.LAYERED, alpha=0.5,
                       fixed_T=True, want_llr=True)
    np.testing.assert_array_equal(fl.llr[0, 0], [0.5, 4.0, 5.5])
    np.testing.assert_array_equal(se.llr[0, 0], [0.5, 4.0, 5.0])


def _random_tree(rng, n_checks, wmin=2, wmax=4):
    """Random tree-shaped Tanner graph: each new check shares exactly one existing variable."""
    rows = []
    nvar = 0
    for j in range(n_checks):
        w = int(rng.integers(wmin, wmax + 1))
        if j == 0:
            vs = list(range(w))
            nvar = w
        else:
            anchor = int(rng.integers(0, nvar))
            vs = [anchor] + list(range(nvar, nvar + w - 1))
            nvar += w - 1
        rows.append(vs)
    h = np.zeros((n_checks, nvar), np.uint8)
    for j, vs in enumerate(rows):
        h[j, vs] = 1
    perm = rng.permutation(nvar)     # scramble variable labels
    return h[:, perm]


def _brute_posteriors(h, s, mu, mode):
    """Exact LLRs ln P(e_i=0|s)/P(e_i=1|s) ('sum') or min-cost differences ('min')."""
    m, n = h.shape
    E = np.array(list(itertools.product([0, 1], repeat=n)), np.int64)
    ok = ((E @ h.T.astype(np.int64)) % 2 == s[None, :]).all(axis=1)
    E = E[ok]
    cost = E @ mu                     # -log-likelihood up to a constant
    out = np.zeros(n)
    for i in range(n):
        c0, c1 = cost[E[:, i] == 0], cost[E[:, i] == 1]
        if mode == "sum":
            a0 = np.log(np.exp(-(c0 - cost.min())).sum())
            a1 = np.log(np.exp(-(c1 - cost.min())).sum())
            out[i] = a0 - a1
        else:
            out[i] = c1.min() - c0.min()
    return out


@pytest.mark.parametrize("schedule", [oracle.FLOODING, oracle.LAYERED])
def test_sum_product_exact_on_trees(schedule):
    """BP is exact on cycle-free graphs (Section III-A): the sum-product posteriors
    equal brute-force marginals."""
    rng = np.random.default_rng(5)
    for trial in range(12):
        h = _random_tree(rng, int(rng.integers(2, 5)))
        n = h.shape[1]
        if n > 14:
            continue
        s = rng.integers(0, 2, h.shape[0]).astype(np.int64)
        mu = rng.uniform(-1.0, 3.0, n)
        res = oracle.decode(h, np.array([0, 0], np.int32), np.array([], np.int32),
                            oracle.pack(s[None, :].astype(np.uint8)), mu, T=30, schedule=schedule,
                            rule=oracle.SPA, fixed_T=True, want_llr=True)
        np.testing.assert_allclose(res.llr[0, 0], _brute_posteriors(h, s, mu, "sum"),
                                   rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("schedule", [oracle.FLOODING, oracle.LAYERED])
def test_min_sum_is_min_cost_on_trees(schedule):
    """Min-sum with alpha = 1 on a tree computes min-cost differences exactly."""
    rng = np.random.default_rng(6)
    for trial in range(12):
        h = _random_tree(rng, int(rng.integers(2, 5)))
        n = h.shape[1]
        if n > 14:
            continue
        s = rng.integers(0, 2, h.shape[0]).astype(np.int64)
        mu = rng.uniform(0.5, 3.0, n)
        res = oracle.decode(h, np.array([0, 0], np.int32), np.array([], np.int32),
                            oracle.pack(s[None, :].astype(np.uint8)), mu, T=30, schedule=schedule,
                            rule=oracle.NMS, alpha=1.0, fixed_T=True, want_llr=True)
        np.testing.assert_allclose(res.llr[0, 0], _brute_posteriors(h, s, mu, "min"),
                                   rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("precision,rtol", [("f64", 1e-12), ("f32", 2e-6)])
def test_sum_product_large_magnitudes(precision, rtol):
    """The tanh rule at magnitudes up to the clamp (the messages of the serial schedule
    on codes with cycles get there).  One check, T = 1, so P_0 = mu_0 + r(c -> v0).
    Weight 2: r = +-phi(phi(|mu_1|)) = +-|mu_1| (phi is its own inverse).  Weight 3:
    2 atanh(tanh(a/2) tanh(b/2)) has the closed form
    min(a, b) - ln(1 + e^-|a-b|) + ln(1 + e^-(a+b)).  Beyond r_max the message is
    clamped."""
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    for a in (0.3, 5.0, 50.0, 500.0, 5000.0, 60000.0):
        for s in (0, 1):
            res = oracle.decode(np.array([[1, 1]], np.uint8), bp, rows, oracle.pack(np.array([[s]], np.uint8)),
                                np.array([1.0, a]), T=1, rule=oracle.SPA, fixed_T=True, want_llr=True,
                                precision=precision)
            assert res.llr[0, 0, 0] == pytest.approx(1.0 + (-a if s else a), rel=rtol)
    for a, b in ((3.0, 4.0), (40.0, 41.5), (800.0, 800.25), (2000.0, 1999.0), (7000.0, 9000.0)):
        res = oracle.decode(np.array([[1, 1, 1]], np.uint8), bp, rows, oracle.pack(np.array([[0]], np.uint8)),
                            np.array([1.0, a, b]), T=1, rule=oracle.SPA, fixed_T=True, want_llr=True,
                            precision=precision)
        expect = min(a, b) - np.log1p(np.exp(-abs(a - b))) + np.log1p(np.exp(-(a + b)))
        assert res.llr[0, 0, 0] == pytest.approx(1.0 + expect, rel=rtol)
    res = oracle.decode(np.array([[1, 1]], np.uint8), bp, rows, oracle.pack(np.array([[0]], np.uint8)),
                        np.array([1.0, 1e6]), T=1, rule=oracle.SPA, fixed_T=True, want_llr=True,
                        precision=precision)
    assert res.llr[0, 0, 0] == 1.0 + 65536.0 and bool(res.clamp[0, 0])


def test_tree_from_a_code_subtree():
    """H_t of a maximal subtree, restricted to its variables, is a tree: sum-product on
    it is exact (the structure Section III-A builds on)."""
    c = codes.bb72()
    lists = oracle.subtree_lists(c.hx, np.arange(36))
    rows = lists[0][:2]     # a prefix of the acceptance order is itself a tree
    sub = c.hx[rows]
    h = sub[:, sub.any(axis=0)]
    rng = np.random.default_rng(9)
    s = rng.integers(0, 2, h.shape[0]).astype(np.int64)
    mu = rng.uniform(0.5, 2.0, h.shape[1])
    res = oracle.decode(h, np.array([0, 0], np.int32), np.array([], np.int32),
                        oracle.pack(s[None, :].astype(np.uint8)), mu, T=10, rule=oracle.SPA,
                        fixed_T=True, want_llr=True)
    np.testing.assert_allclose(res.llr[0, 0], _brute_posteriors(h, s, mu, "sum"), atol=1e-9)


def test_zero_syndrome_stops_at_iteration_zero():
    c = codes.bb72()
    bp, rows = _one_basis(c.hx, [1, 2])
    res = oracle.decode(c.hx, bp, rows, np.zeros((3, 1), np.uint64), np.full(72, 2.0), T=20)
    assert (res.K == 0).all() and res.conv.all() and (res.corr == 0).all() and (res.chosen == 0).all()


def _chain():
    """Two weight-2 checks on three variables: c0 = {v0, v1}, c1 = {v1, v2}."""
    return np.array([[1, 1, 0], [0, 1, 1]], np.uint8)


@pytest.mark.parametrize("schedule", [oracle.FLOODING, oracle.LAYERED])
def test_halting_iteration_two_on_a_chain(schedule):
    """Halting rule of Section II-B (stop at the first t whose hard decision meets
    the syndrome).  Chain c0 = {v0, v1}, c1 = {v1, v2}, s = (0, 1), mu = (2, 1, 4),
    alpha = 1, worked by hand.  Flooding:
      t=1: q = mu; r(c0->v0) = 1, r(c0->v1) = 2, r(c1->v1) = -4, r(c1->v2) = -1
           P = (3, -1, 3), e = (0, 1, 0): c0 has parity 1 != 0, not met;
      t=2: q(v1->c0) = 1 - 4 = -3, q(v1->c1) = 1 + 2 = 3
           r(c0->v0) = -3, r(c0->v1) = 2, r(c1->v1) = -4, r(c1->v2) = -3
           P = (-1, -1, 1), e = (1, 1, 0): parities (0, 1) = s, met: K = 2.
    Serial (rows in order, r = 0 before the first sweep):
      t=1: c0 sees q(v1) = 1 + 0: r(c0->v0) = 1, r(c0->v1) = 2; c1 sees
           q(v1) = 1 + 2 = 3: r(c1->v1) = -4, r(c1->v2) = -3; P = (3, -1, 1),
           e = (0, 1, 0), not met;
      t=2: c0 sees q(v1) = -3: r(c0->v0) = -3, r(c0->v1) = 2; c1 as before;
           P = (-1, -1, 1), met: K = 2."""
    h = _chain()
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    syn = oracle.pack(np.array([[0, 1]], np.uint8))
    res = oracle.decode(h, bp, rows, syn, np.array([2.0, 1.0, 4.0]), T=10, schedule=schedule, alpha=1.0,
                        want_llr=True)
    assert int(res.K[0, 0]) == 2 and bool(res.conv[0, 0])
    np.testing.assert_array_equal(res.llr[0, 0], [-1.0, -1.0, 1.0])
    np.testing.assert_array_equal(oracle.unpack(res.corr, 3)[0], [1, 1, 0])
    assert int(res.chosen[0]) == 0
    # one iteration short of K: the same decoder with T = 1 does not converge and
    # reports the t = 1 state
    r1 = oracle.decode(h, bp, rows, syn, np.array([2.0, 1.0, 4.0]), T=1, schedule=schedule, alpha=1.0,
                       want_llr=True)
    assert int(r1.K[0, 0]) == 1 and not bool(r1.conv[0, 0]) and int(r1.chosen[0]) == -1
    expect_t1 = [3.0, -1.0, 3.0] if schedule == oracle.FLOODING else [3.0, -1.0, 1.0]
    np.testing.assert_array_equal(r1.llr[0, 0], expect_t1)
    assert not r1.corr.any()


def test_halting_iteration_separates_the_schedules():
    """The chain with its rows swapped, c0 = {v1, v2}, c1 = {v0, v1}, s = (1, 0),
    mu = (2, 1, 4), alpha = 1.  Serial, t=1: c0 sees q = (1, 4): r(c0->v1) = -4,
    r(c0->v2) = -1; c1 sees q(v0) = 2, q(v1) = 1 - 4 = -3: r(c1->v0) = -3,
    r(c1->v1) = 2; P = (-1, -1, 3), e = (1, 1, 0) meets s: K = 1.  Flooding needs
    the second iteration as above (the same graph): K = 2."""
    h = _chain()[::-1].copy()
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    syn = oracle.pack(np.array([[1, 0]], np.uint8))
    mu = np.array([2.0, 1.0, 4.0])
    se = oracle.decode(h, bp, rows, syn, mu, T=10, schedule=oracle.LAYERED, alpha=1.0, want_llr=True)
    fl = oracle.decode(h, bp, rows, syn, mu, T=10, schedule=oracle.FLOODING, alpha=1.0, want_llr=True)
    assert int(se.K[0, 0]) == 1 and bool(se.conv[0, 0])
    np.testing.assert_array_equal(se.llr[0, 0], [-1.0, -1.0, 3.0])
    assert int(fl.K[0, 0]) == 2 and bool(fl.conv[0, 0])
    np.testing.assert_array_equal(fl.llr[0, 0], [-1.0, -1.0, 1.0])


@pytest.mark.parametrize("schedule", [oracle.FLOODING, oracle.LAYERED])
def test_halting_iteration_one_and_never(schedule):
    """One check {v0, v1}, s = 1, mu = (1, 3).  After one iteration r(->v0) = -3 alpha,
    r(->v1) = -alpha, and every later iteration repeats it (each variable has one
    check, so q = mu).  alpha = 1/2: P = (-0.5, 2.5), e = (1, 0) meets s at t = 1.
    alpha = 1/4: P = (0.25, 2.75), e = 0 never meets s: not converged, K = T."""
    h = np.array([[1, 1]], np.uint8)
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    syn = oracle.pack(np.array([[1]], np.uint8))
    mu = np.array([1.0, 3.0])
    a = oracle.decode(h, bp, rows, syn, mu, T=7, schedule=schedule, alpha=0.5, want_llr=True)
    assert int(a.K[0, 0]) == 1 and bool(a.conv[0, 0])
    np.testing.assert_array_equal(a.llr[0, 0], [-0.5, 2.5])
    b = oracle.decode(h, bp, rows, syn, mu, T=7, schedule=schedule, alpha=0.25, want_llr=True)
    assert int(b.K[0, 0]) == 7 and not bool(b.conv[0, 0]) and int(b.chosen[0]) == -1
    np.testing.assert_array_equal(b.llr[0, 0], [0.25, 2.75])


def test_halting_with_a_zero_posterior():
    """A posterior of exactly 0 decides e = 0 (ties go to 0, Section II-B's hard
    decision).  Chain, s = (0, 1), mu = (2, 1, 4), alpha = 1/2, flooding:
      t=1: r(c0->v0) = 0.5, r(c0->v1) = 1, r(c1->v1) = -2, r(c1->v2) = -0.5,
           P = (2.5, 0, 3.5), e = 0, c1 unmet;
      t=2: q(v1->c0) = -1, q(v1->c1) = 2: r(c0->v0) = -0.5, r(c0->v1) = 1,
           r(c1->v1) = -2, r(c1->v2) = -1, P = (1.5, 0, 3), e = 0;
      later iterations repeat t=2: never converges, K = T."""
    h = _chain()
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    syn = oracle.pack(np.array([[0, 1]], np.uint8))
    mu = np.array([2.0, 1.0, 4.0])
    r1 = oracle.decode(h, bp, rows, syn, mu, T=1, alpha=0.5, want_llr=True)
    np.testing.assert_array_equal(r1.llr[0, 0], [2.5, 0.0, 3.5])
    r = oracle.decode(h, bp, rows, syn, mu, T=9, alpha=0.5, want_llr=True)
    assert int(r.K[0, 0]) == 9 and not bool(r.conv[0, 0])
    np.testing.assert_array_equal(r.llr[0, 0], [1.5, 0.0, 3.0])
    assert not oracle.unpack(r.cand[0, 0], 3).any()


def test_fixed_T_reports_the_first_halting_iteration():
    """Diagnostic fixed-T mode: K is the first iteration whose decision met the
    syndrome, the posterior is the state after T.  Chain as above (K = 2, a fixed
    point from t = 2 on), and the single check with alpha = 1/2 (K = 1)."""
    h = _chain()
    bp, rows = np.array([0, 0], np.int32), np.array([], np.int32)
    syn = oracle.pack(np.array([[0, 1]], np.uint8))
    r = oracle.decode(h, bp, rows, syn, np.array([2.0, 1.0, 4.0]), T=6, alpha=1.0, fixed_T=True, want_llr=True)
    assert int(r.K[0, 0]) == 2 and bool(r.conv[0, 0])
    np.testing.assert_array_equal(r.llr[0, 0], [-1.0, -1.0, 1.0])


# ------------------------------------------------------------------ representations: subtree order

def _alg2_reference(h, perm):
    """Algorithm 2 written again for this test from the paper's description
    (Section III-A): roots in pi order; from a root, checks are examined first in,
    first out; a check joins the growing subtree when at most one of its
    variables is already covered (and it is still unassigned), then its
    variables are covered and their untested unassigned checks queued in
    ascending order.  Covered/tested marks start afresh for each root.  Returns
    the subtrees as row lists in acceptance order."""
    from collections import deque
    m, n = h.shape
    rows_of = [list(np.nonzero(h[j])[0]) for j in range(m)]
    checks_of = [list(np.nonzero(h[:, v])[0]) for v in range(n)]
    owner = [None] * m
    out = []
    for root in perm:
        if owner[root] is not None:
            continue
        tree = []
        covered, tested = set(), set()
        q = deque([root])
        while q:
            u = q.popleft()
            tested.add(u)
            if owner[u] is not None or sum(v in covered for v in rows_of[u]) > 1:
                continue
            owner[u] = len(out)
            tree.append(int(u))
            for v in rows_of[u]:
                covered.add(v)
                q.extend(c for c in checks_of[v] if c not in tested and owner[c] is None)
        out.append(tree)
    return out


def test_alg2_reference_reproduces_fig2():
    h, perm, cs_expect, subs = _read_fig2()
    got = _alg2_reference(h, perm)
    assert got == [subs[s] for s in sorted(subs)]


@pytest.mark.parametrize("factory,L", [(codes.bb72, 4), (codes.bb144, 16), (codes.bb288, 32)])
def test_subtree_mode_selection_order(factory, L):
    """Representations of the subtrees mode: the first L distinct subtrees (as row
    sets) met while walking pi_0, pi_1, ... in discovery order, each with its rows
    in acceptance order.  The expected list comes from the reference Algorithm 2
    above, not from the oracle."""
    c = factory()
    for h in (c.hx, c.hz):
        perms = check_permutations(h.shape[0], 8, seed=0)
        expect, seen = [], set()
        for perm in perms:
            for t in _alg2_reference(h, perm):
                key = frozenset(t)
                if key not in seen and len(expect) < L:
                    seen.add(key)
                    expect.append(t)
        bp, rows = oracle.build_bases(h, "subtrees", L, perms)
        got = [rows[bp[l]:bp[l + 1]].tolist() for l in range(L)]
        assert got == expect


def test_ramp_mode_prefixes():
    """Ramp mode: representation l appends the first round(l m / (L - 1)) rows (halves
    up) of pi_l's acceptance order (the reference Algorithm 2's subtrees joined)."""
    c = codes.bb288()
    h = c.hz
    L = 32
    perms = check_permutations(h.shape[0], L, seed=0)
    bp, rows = oracle.build_bases(h, "ramp", L, perms)
    m = h.shape[0]
    for l in range(L):
        r = (2 * l * m + (L - 1)) // (2 * (L - 1))
        joined = [x for t in _alg2_reference(h, perms[l]) for x in t]
        assert rows[bp[l]:bp[l + 1]].tolist() == joined[:r]


# ------------------------------------------------------------------ list decision

def test_decision_rules_worked_example():
    """List with candidate A (weight 2) from bases 0, 2, 3 and B (weight 1) from basis 1:
    least weight picks B (basis 1); FWS scores A 3/3 = 1 > B 1/2 and picks basis 0."""
    A = oracle.pack(np.array([[1, 1, 0, 0]], np.uint8))[0]
    B = oracle.pack(np.array([[0, 0, 1, 0]], np.uint8))[0]
    cand = np.array([[A, B, A, A]], np.uint64)
    conv = np.array([[1, 1, 1, 1]], bool)
    assert oracle.select(cand, conv, oracle.MIN_WEIGHT)[0] == 1
    assert oracle.select(cand, conv, oracle.FWS)[0] == 0
    # ties: equal weights -> smaller basis index; nothing converged -> -1
    C = oracle.pack(np.array([[0, 1, 0, 0]], np.uint8))[0]
    cand2 = np.array([[A, C, B, C]], np.uint64)
    assert oracle.select(cand2, np.array([[0, 1, 1, 1]], bool), oracle.MIN_WEIGHT)[0] == 1
    # FWS: C twice (2/2 = 1) beats B once (1/2)
    assert oracle.select(cand2, np.array([[0, 1, 1, 1]], bool), oracle.FWS)[0] == 1
    assert oracle.select(cand2, np.zeros((1, 4), bool), oracle.FWS)[0] == -1
    assert oracle.select(cand2, np.zeros((1, 4), bool), oracle.MIN_WEIGHT)[0] == -1


# ------------------------------------------------------------------ small codes, brute force

def _stabilizer_group(h):
    return _span(h)


@pytest.mark.parametrize("factory", [codes.steane7, codes.surface13, codes.toric18])
def test_small_codes_against_brute_force(factory):
    """On n <= 18: every accepted candidate meets its syndrome; the chosen weight is at
    least the brute-force minimum weight; failure flags equal stabilizer-group
    membership of the residual."""
    c = factory()
    n = c.n
    perms_x = check_permutations(c.hx.shape[0], 4, seed=2)
    perms_z = check_permutations(c.hz.shape[0], 4, seed=2)
    ex, ez, sx, sz = oracle.sample(c.hx, c.hz, 3, 0.12, 0, 300)
    mu = np.full(n, oracle.prior_llr(0.12))
    all_e = np.array(list(itertools.product([0, 1], repeat=n)), np.int64)
    for h, stab, perms, syn, err in ((c.hz, c.hx, perms_z, sx, ex), (c.hx, c.hz, perms_x, sz, ez)):
        L = 2
        bp, rows = oracle.build_bases(h, "ramp", L, perms)
        res = oracle.decode(h, bp, rows, syn, mu, T=15, alpha=0.875)
        sb = oracle.unpack(syn, h.shape[0]).astype(np.int64)
        cb = oracle.unpack(res.cand, n).astype(np.int64)
        hh = h.astype(np.int64)
        for s in range(syn.shape[0]):
            for l in range(L):
                if res.conv[s, l]:
                    np.testing.assert_array_equal((cb[s, l] @ hh.T) % 2, sb[s])
        synd_all = (all_e @ hh.T) % 2
        group = _stabilizer_group(stab)
        fails = oracle.failures(stab, err, res.corr)
        eb = oracle.unpack(err, n)
        corr_b = oracle.unpack(res.corr, n)
        for s in range(syn.shape[0]):
            if res.chosen[s] >= 0:
                wmin = all_e[(synd_all == sb[s]).all(axis=1)].sum(axis=1).min()
                assert corr_b[s].sum() >= wmin
            resid = (eb[s] ^ corr_b[s]).astype(np.uint8)
            assert fails[s] == (resid.tobytes() not in group)


def test_failure_flags_known_cases():
    """Steane: a stabilizer residual is no failure; the all-ones logical is one."""
    c = codes.steane7()
    err = oracle.pack(np.array([[1, 0, 1, 0, 1, 0, 1], [1, 1, 1, 1, 1, 1, 1], [0] * 7], np.uint8))
    corr = oracle.pack(np.zeros((3, 7), np.uint8))
    np.testing.assert_array_equal(oracle.failures(c.hx, err, corr), [False, True, False])


def test_general_row_not_in_rowspace_rejected():
    c = codes.steane7()
    bp = np.array([0, 1], np.int32)
    rows = np.array([-1], np.int32)
    with pytest.raises(oracle.OracleError) as ei:
        oracle.decode(c.hx, bp, rows, np.zeros((1, 1), np.uint64), np.full(7, 2.0), T=3,
                      explicit={0: np.array([1, 0, 0, 0, 0, 0, 0], np.uint8)})
    assert ei.value.status == oracle.ORC_ENOTINROWSPACE
    # a sum of two rows is accepted and its syndrome bit is the sum of theirs
    row = (c.hx[0] ^ c.hx[1]).astype(np.uint8)
    res = oracle.decode(c.hx, bp, rows, oracle.pack(np.array([[1, 0, 0]], np.uint8)),
                        np.full(7, 2.0), T=1, fixed_T=True, want_llr=True, alpha=1.0,
                        explicit={0: row})
    haug = np.concatenate([c.hx, row[None]], 0).astype(np.int64)
    saug = np.array([1, 0, 0, 1])
    np.testing.assert_allclose(res.llr[0, 0], 2.0 + 2.0 * ((1 - 2 * saug) @ haug))


def test_f32_build_is_single_precision():
    assert oracle._lib("f32").orc_real_bytes() == 4
    assert oracle._lib("f64").orc_real_bytes() == 8
