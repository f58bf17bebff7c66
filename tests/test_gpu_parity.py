"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

* noise and syndromes: bit-exact;
* normalized min-sum: bit-exact against the single-precision oracle build on every
  per-representation output (hard decisions, iteration counts, convergence flags,
  posterior LLR bit patterns), the list decision and the failure flags;
* against the FP64 oracle: decisions may differ only on instances whose FP64 run
  came within 1e-3 of a sign flip (counted and printed), and fixed-T posteriors of
  those that agree on every decision stay within 1e-4 * max(1, |LLR|);
* sum-product: FP64 oracle within tolerance on cycle-free graphs (where BP is exact);
* batched (persistent) form: bit-identical to the plain form.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import codes
from workloads.configs import WORKLOADS

from .common import bases_for, f32, tie_shots

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_14170_amd as m
    return m


def make_decoder(pk, code, wl, T=None, **kw):
    bx = bases_for(code.hx, wl, oracle.build_bases)
    bz = bases_for(code.hz, wl, oracle.build_bases)
    dec = pk.Decoder(code.hx, code.hz, bx, bz, wl.T if T is None else T, alpha=wl.alpha, **kw)
    return dec, bx, bz


def words(t):
    return t.detach().cpu().numpy().view(np.uint64)


# ------------------------------------------------------------------------ sampler

@pytest.mark.parametrize("key,p,shot0,shots", [
    ("bb72_L4_T20", 0.05, 0, 1000),
    ("bb144_L16_T50", 0.08, 12345, 777),          # ragged tail, offset start
    ("qc882_L64_T100", 0.03, 10**9, 130),
])
def test_sampler_bit_exact(pk, key, p, shot0, shots):
    wl = WORKLOADS[key]
    code = wl.code()
    bases = (np.zeros(2, np.int32), np.zeros(0, np.int32))
    say(f"sampler {key} p={p} shot0={shot0} shots={shots}")
    dec = pk.Decoder(code.hx, code.hz, bases, bases, 1, max_batch=shots)
    ex, ez, sx, sz = dec.sample(wl.seed, p, shot0, shots)
    torch.cuda.synchronize()
    oex, oez, osx, osz = oracle.sample(code.hx, code.hz, wl.seed, p, shot0, shots)
    np.testing.assert_array_equal(words(ex), oex)
    np.testing.assert_array_equal(words(ez), oez)
    np.testing.assert_array_equal(words(sx), osx)
    np.testing.assert_array_equal(words(sz), osz)
    dec.close()


# ------------------------------------------------------------------------ NMS flooding, bit-exact vs FP32 oracle

def _detail_vs_oracle(pk, dec, code, bx, bz, wl, p, shot0, shots, precision, fixed_T=False):
    ex, ez, sx, sz = dec.sample(wl.seed, p, shot0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = []
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
        torch.cuda.synchronize()
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), dec.T, alpha=wl.alpha,
                            fixed_T=fixed_T, want_llr=True, precision=precision)
        ks = kstat.cpu().numpy().view(np.uint16)
        out.append((part, words(cand), (ks & 0x7FFF).astype(np.int32), (ks >> 15).astype(bool),
                    llr.cpu().numpy(), ref))
    return out


@pytest.mark.parametrize("key,p,shots", [("bb72_L4_T20", 0.05, 10000), ("bb144_L16_T50", 0.04, 1500),
                                         ("bb144_L16_T50", 0.08, 600)])
def test_nms_flooding_bit_exact_fp32(pk, key, p, shots):
    wl = WORKLOADS[key]
    code = wl.code()
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"nms flooding fp32 bit-exact {key} p={p} shots={shots}")
    for part, cand, K, conv, llr, ref in _detail_vs_oracle(pk, dec, code, bx, bz, wl, p, 0, shots, "f32"):
        np.testing.assert_array_equal(K, ref.K, err_msg=f"part {part} iterations")
        np.testing.assert_array_equal(conv, ref.conv, err_msg=f"part {part} convergence")
        np.testing.assert_array_equal(cand, ref.cand, err_msg=f"part {part} hard decisions")
        np.testing.assert_array_equal(llr.view(np.uint32), ref.llr.astype(np.float32).view(np.uint32),
                                      err_msg=f"part {part} posterior bits")
        say(f"  part {part}: mean K {K.mean():.3f}, converged {conv.mean():.4f}")
    dec.close()


def test_nms_fixed_T_fp32_and_fp64(pk):
    """Fixed-T diagnostic: bit-exact vs FP32 oracle; vs FP64 oracle the decisions differ
    only on tie-prone instances and agreeing instances keep |dLLR| <= 1e-4 max(1, |LLR|)."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p = 400, 0.06
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, fixed_T=True)
    say(f"fixed-T bb144 p={p} shots={shots}")
    res32 = _detail_vs_oracle(pk, dec, code, bx, bz, wl, p, 5000, shots, "f32", fixed_T=True)
    for part, cand, K, conv, llr, ref in res32:
        np.testing.assert_array_equal(cand, ref.cand)
        np.testing.assert_array_equal(K, ref.K)
        np.testing.assert_array_equal(llr.view(np.uint32), ref.llr.astype(np.float32).view(np.uint32))
    res64 = _detail_vs_oracle(pk, dec, code, bx, bz, wl, p, 5000, shots, "f64", fixed_T=True)
    total = ties = diff = 0
    for part, cand, K, conv, llr, ref in res64:
        same = (cand == ref.cand).all(axis=-1) & (K == ref.K) & (conv == ref.conv)
        tie = tie_shots(ref.margin)
        total += same.size
        ties += int(tie.sum())
        diff += int((~same).sum())
        assert not (~same & ~tie).any(), "decision differs on a non-tie instance"
        ok = same & ~ref.clamp
        err = np.abs(llr.astype(np.float64) - ref.llr)[ok]
        bound = 1e-4 * np.maximum(1.0, np.abs(ref.llr[ok]))
        frac = float((err <= bound).mean())
        say(f"  part {part}: instances {same.size}, differing {int((~same).sum())}, tie-prone {int(tie.sum())}, "
            f"LLR within tolerance {frac:.6f}")
    say(f"  fp64: {diff} of {total} instances differ, all among {ties} tie-prone")
    dec.close()


def test_decode_select_failures_bit_exact(pk):
    """The whole plain path: decisions, chosen representation, convergence mask and
    failure flags equal the FP32 oracle's."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p = 2000, 0.06
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"decode+select+failures bb144 p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(wl.seed, p, 777, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode(sx, sz, prior, prior)
    fail = dec.failures(ex, ez, out["corr_x"], out["corr_z"])
    torch.cuda.synchronize()
    fail_ref = np.zeros(shots, np.uint8)
    for part, h, (bp, rows), syn, err, stab in ((0, code.hz, bz, sx, ex, code.hx),
                                                 (1, code.hx, bx, sz, ez, code.hz)):
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, alpha=wl.alpha,
                            precision="f32")
        tag = "x" if part == 0 else "z"
        np.testing.assert_array_equal(words(out[f"corr_{tag}"]), ref.corr)
        np.testing.assert_array_equal(out[f"basis_{tag}"].cpu().numpy(), ref.chosen)
        mask = (ref.conv.astype(np.uint64) << np.arange(wl.L, dtype=np.uint64)).sum(axis=1).astype(np.uint64)
        np.testing.assert_array_equal(words(out[f"conv_{tag}"]), mask)
        fail_ref |= oracle.failures(stab, words(err), ref.corr).astype(np.uint8) << part
    np.testing.assert_array_equal(fail.cpu().numpy(), fail_ref)
    say(f"  LER {float((fail_ref != 0).mean()):.4f}")
    dec.close()


def test_batched_bit_identical_to_plain(pk):
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p = 5000, 0.08
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"batched vs plain bb144 p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(3, p, 0, shots)
    prior = torch.full((code.n,), f32(oracle.prior_llr(p)), dtype=torch.float32, device="cuda")
    a = dec.decode(sx, sz, prior, prior)
    b = dec.decode_batched(sx, sz, prior, prior)
    torch.cuda.synchronize()
    for k in a:
        np.testing.assert_array_equal(a[k].cpu().numpy(), b[k].cpu().numpy(), err_msg=k)
    dec.close()


def test_per_shot_priors(pk):
    """prior_per_shot = 1 (non-uniform soft priors) matches the oracle bit for bit."""
    wl = WORKLOADS["bb72_L4_T20"]
    code = wl.code()
    shots = 300
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"per-shot priors bb72 shots={shots}")
    ex, ez, sx, sz = dec.sample(9, 0.05, 0, shots)
    rng = np.random.default_rng(4)
    pri = rng.uniform(0.5, 5.0, (shots, code.n)).astype(np.float32)
    pt = torch.from_numpy(pri).cuda()
    cand, kstat, _ = dec.decode_detail(0, sx, pt)
    torch.cuda.synchronize()
    ref = oracle.decode(code.hz, *bz, words(sx), pri.astype(np.float64), wl.T, alpha=wl.alpha, precision="f32")
    np.testing.assert_array_equal(words(cand), ref.cand)
    np.testing.assert_array_equal(kstat.cpu().numpy().view(np.uint16) & 0x7FFF, ref.K)
    dec.close()


# ------------------------------------------------------------------------ sum-product

def test_spa_exact_on_trees(pk):
    """On a cycle-free Tanner graph, GPU sum-product posteriors equal the FP64 oracle's
    (which equal exact marginals) within 1e-4 * max(1, |LLR|)."""
    from .test_oracle_pins import _random_tree
    rng = np.random.default_rng(21)
    bases = (np.zeros(2, np.int32), np.zeros(0, np.int32))
    for trial in range(6):
        h = _random_tree(rng, int(rng.integers(3, 7)), wmin=3, wmax=5)
        n = h.shape[1]
        say(f"spa tree trial {trial} n={n}")
        dec = pk.Decoder(h, _commuting_pair(h), bases, bases, 30, rule=pk.SPA, fixed_T=True, max_batch=64)
        s = rng.integers(0, 2, (64, h.shape[0])).astype(np.uint8)
        syn = torch.from_numpy(oracle.pack(s).view(np.int64)).cuda()
        mu = rng.uniform(-1.0, 3.0, n).astype(np.float32)
        cand, kstat, llr = dec.decode_detail(1, syn, torch.from_numpy(mu).cuda(), want_llr=True)
        torch.cuda.synchronize()
        ref = oracle.decode(h, np.array([0, 0], np.int32), np.array([], np.int32), oracle.pack(s),
                            mu.astype(np.float64), 30, rule=oracle.SPA, fixed_T=True, want_llr=True)
        got = llr.cpu().numpy()[:, 0, :].astype(np.float64)
        exp = ref.llr[:, 0, :]
        err = np.abs(got - exp) / np.maximum(1.0, np.abs(exp))
        say(f"  max relative LLR error {err.max():.3e}")
        assert np.all(err <= 1e-4)
        dec.close()


def _commuting_pair(h):
    """A weight-2 row on two variables with identical columns in h (it commutes with
    every row of h); the last check of a random tree of weight >= 3 has two leaves."""
    n = h.shape[1]
    for a in range(n):
        for b in range(a + 1, n):
            if (h[:, a] == h[:, b]).all():
                r = np.zeros((1, n), np.uint8)
                r[0, [a, b]] = 1
                return r
    raise AssertionError("no identical column pair")
