"""CPU checks of the C ABI: the library loads, exports every declared symbol, its
host-only entry points (Algorithm 2, representation assembly) match the oracle
exactly, and argument validation rejects bad inputs before touching a device."""

import ctypes

import numpy as np
import pytest

import oracle
import paper_2605_14170_amd as pk
from paper_2605_14170_amd import _lib
from workloads import codes, check_permutations

from .common import header_symbols


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    declared = header_symbols()
    assert len(declared) >= 14
    for name in declared:
        assert hasattr(lib, name), name
    assert set(_lib.EXPORTED) <= set(declared)


@pytest.mark.parametrize("factory", [codes.bb72, codes.bb144, codes.bb288, codes.qc882,
                                     codes.steane7, codes.toric18])
def test_subtrees_match_oracle(factory):
    c = factory()
    for h in (c.hx, c.hz):
        for perm in check_permutations(h.shape[0], 4, seed=5):
            a = pk.subtrees(h, perm)
            b = oracle.subtrees(h, perm)
            np.testing.assert_array_equal(a[0], b[0])
            np.testing.assert_array_equal(a[1], b[1])
            assert a[2] == b[2]


def test_fig2_through_library():
    cs, order, ns = pk.subtrees(codes.fig2_matrix(), [0, 3, 1, 2])
    assert list(cs) == [1, 2, 1, 2] and list(order) == [0, 2, 3, 1] and ns == 2


@pytest.mark.parametrize("factory,mode,L", [(codes.bb72, "subtrees", 4), (codes.bb144, "subtrees", 16),
                                            (codes.bb288, "ramp", 32), (codes.qc882, "ramp", 64)])
def test_bases_match_oracle(factory, mode, L):
    c = factory()
    for h in (c.hx, c.hz):
        perms = check_permutations(h.shape[0], max(L, 8), seed=0)
        a = pk.build_bases(h, mode, L, perms)
        b = oracle.build_bases(h, mode, L, perms)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def _create(hx, hz, bx, bz, T=5, **kw):
    return pk.Decoder(hx, hz, bx, bz, T, **kw)


def _plain_bases(L=1):
    return (np.zeros(L + 1, np.int32), np.zeros(0, np.int32))


def test_create_rejects_noncommuting():
    c = codes.steane7()
    hz = c.hz.copy()
    hz[0, 0] ^= 1
    with pytest.raises(pk.MbbpError) as ei:
        _create(c.hx, hz, _plain_bases(), _plain_bases())
    assert ei.value.status == -1 and "H_X H_Z^T" in str(ei.value)


def test_create_rejects_bad_shapes_and_rows():
    c = codes.steane7()
    with pytest.raises(pk.MbbpError) as ei:
        _create(c.hx[:, :6], c.hz, _plain_bases(), _plain_bases())
    assert ei.value.status == -1
    # basis row out of range
    with pytest.raises(pk.MbbpError) as ei:
        _create(c.hx, c.hz, (np.array([0, 1], np.int32), np.array([7], np.int32)), _plain_bases())
    assert ei.value.status == -1
    # L > 64
    with pytest.raises(pk.MbbpError) as ei:
        _create(c.hx, c.hz, _plain_bases(65), _plain_bases(65))
    assert ei.value.status == -5
    # negative T
    with pytest.raises(pk.MbbpError) as ei:
        _create(c.hx, c.hz, _plain_bases(), _plain_bases(), T=-1)
    assert ei.value.status == -1


def test_create_rejects_row_outside_rowspace():
    c = codes.steane7()
    extra = np.zeros((1, 7), np.uint8)
    extra[0, :3] = 1   # weight 3, not in the Hamming row space (min weight there is 4)
    with pytest.raises(pk.MbbpError) as ei:
        _create(c.hx, c.hz, (np.array([0, 1], np.int32), np.array([-1], np.int32)), _plain_bases(),
                extra_hx=extra)
    assert ei.value.status == -2


def test_create_rejects_heavy_rows():
    # a 9-column all-ones row: weight 9 > 8 (H_Z chosen to commute)
    hx = np.ones((1, 10), np.uint8)
    hx[0, 9] = 0
    hz = np.zeros((1, 10), np.uint8)
    hz[0, [0, 1]] = 1
    with pytest.raises(pk.MbbpError) as ei:
        _create(hx, hz, _plain_bases(), _plain_bases())
    assert ei.value.status == -5


def test_build_bases_errors():
    c = codes.bb72()
    perms = check_permutations(36, 2, seed=0)
    with pytest.raises(pk.MbbpError):
        pk.build_bases(c.hx, "subtrees", 40, perms)       # not enough distinct subtrees
    with pytest.raises(pk.MbbpError):
        pk.build_bases(c.hx, "ramp", 4, perms)            # ramp needs a permutation per basis
    bad = perms.copy()
    bad[0, 0] = bad[0, 1]
    with pytest.raises(pk.MbbpError):
        pk.subtrees(c.hx, bad[0])


def test_last_error_is_thread_local_text():
    lib = _lib.lib()
    with pytest.raises(pk.MbbpError):
        pk.subtrees(codes.bb72().hx, np.zeros(36, np.int32))
    assert b"permutation" in lib.mbbp_last_error()


def test_set_noise_validates_arguments():
    """mbbp_set_noise: a null context and an unknown model are MBBP_EINVAL (host
    checks only, no device call)."""
    lib = _lib.lib()
    assert lib.mbbp_set_noise(None, 0) == -1
    assert b"null ctx" in lib.mbbp_last_error()
    assert pk.DEPOLARIZING == 0 and pk.X_ONLY == 1 and oracle.BSC_X == pk.X_ONLY


def test_partition_bases():
    """Table II inputs: tree bases are the partition's subtrees in acceptance order;
    matched random bases have the same sizes, distinct in-range rows, are seeded
    and differ between partitions."""
    import oracle
    from workloads import codes
    from workloads.partitions import matched_random_bases, tree_bases
    from workloads.perms import check_permutations
    h = codes.bb288().hz
    m = h.shape[0]
    perms = check_permutations(m, 3, seed=0)
    subs = oracle.subtree_lists(h, perms[1])
    bp, rows = tree_bases(subs)
    assert [rows[bp[i]:bp[i + 1]].tolist() for i in range(len(subs))] == subs
    bp2, rows2 = tree_bases(subs, count=len(subs) + 3)
    assert rows2[bp2[len(subs)]:].tolist() == [x for s in subs[:3] for x in s]
    rb, rr = matched_random_bases(subs, m, seed=5, k=1)
    np.testing.assert_array_equal(np.diff(rb), [len(s) for s in subs])
    for i in range(len(subs)):
        r = rr[rb[i]:rb[i + 1]]
        assert len(set(r.tolist())) == len(r) and (r >= 0).all() and (r < m).all()
    rb_again, rr_again = matched_random_bases(subs, m, seed=5, k=1)
    np.testing.assert_array_equal(rr, rr_again)
    _, rr_other = matched_random_bases(subs, m, seed=5, k=2)
    assert rr_other.tolist() != rr.tolist()
