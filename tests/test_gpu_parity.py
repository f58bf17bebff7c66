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


@pytest.mark.parametrize("key,p,shot0,shots", [("bb144_L16_T50", 0.07, 999, 513), ("bb72_L4_T20", 0.5, 0, 64)])
def test_sampler_x_only_bit_exact(pk, key, p, shot0, shots):
    """X-only noise (mbbp_set_noise): errors and syndromes equal the oracle's."""
    wl = WORKLOADS[key]
    code = wl.code()
    bases = (np.zeros(2, np.int32), np.zeros(0, np.int32))
    say(f"sampler x-only {key} p={p} shot0={shot0} shots={shots}")
    dec = pk.Decoder(code.hx, code.hz, bases, bases, 1, max_batch=shots)
    dec.set_noise(pk.X_ONLY)
    ex, ez, sx, sz = dec.sample(wl.seed, p, shot0, shots)
    torch.cuda.synchronize()
    oex, oez, osx, osz = oracle.sample(code.hx, code.hz, wl.seed, p, shot0, shots, oracle.BSC_X)
    np.testing.assert_array_equal(words(ex), oex)
    np.testing.assert_array_equal(words(ez), oez)
    np.testing.assert_array_equal(words(sx), osx)
    np.testing.assert_array_equal(words(sz), osz)
    assert not oez.any()
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


def test_nms_fixed_T_fp32_and_short_horizon_fp64(pk):
    """Fixed-T diagnostic.  Bit-exact vs the FP32 oracle at T = 50.  Against the FP64
    oracle at a horizon of T = 5 iterations every hard decision agrees except on
    tie-prone instances (FP64 margin < 1e-3), and every posterior is within
    1e-4 * max(1, |LLR|)."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p = 400, 0.06
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, fixed_T=True)
    say(f"fixed-T bb144 p={p} shots={shots}")
    for part, cand, K, conv, llr, ref in _detail_vs_oracle(pk, dec, code, bx, bz, wl, p, 5000, shots, "f32",
                                                            fixed_T=True):
        np.testing.assert_array_equal(cand, ref.cand)
        np.testing.assert_array_equal(K, ref.K)
        np.testing.assert_array_equal(llr.view(np.uint32), ref.llr.astype(np.float32).view(np.uint32))
    dec.close()
    dec5, _, _ = make_decoder(pk, code, wl, T=5, max_batch=shots, fixed_T=True)
    for part, cand, K, conv, llr, ref in _detail_vs_oracle(pk, dec5, code, bx, bz, wl, p, 5000, shots, "f64",
                                                            fixed_T=True):
        same = (cand == ref.cand).all(axis=-1) & (K == ref.K) & (conv == ref.conv)
        tie = tie_shots(ref.margin)
        assert not (~same & ~tie).any(), "decision differs from FP64 on a non-tie instance"
        err = np.abs(llr.astype(np.float64) - ref.llr) / np.maximum(1.0, np.abs(ref.llr))
        say(f"  part {part}: T=5 vs FP64: differing {int((~same).sum())} of {same.size} (ties {int(tie.sum())}), "
            f"max relative LLR error {err.max():.2e}")
        assert err.max() <= 1e-4
    dec5.close()


def test_full_T_fp64_statistics(pk):
    """At T = 50 FP32 and FP64 BP trajectories separate on a few per cent of
    instances (chaotic, mostly non-converging ones), so there the comparison is
    statistical: the GPU's logical error rate lies inside the FP64 oracle's Wilson
    95% interval.  The differing-instance count is printed."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p = 1500, 0.06
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"full-T FP64 statistics bb144 p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(wl.seed, p, 40000, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode(sx, sz, prior, prior)
    fail = dec.failures(ex, ez, out["corr_x"], out["corr_z"]).cpu().numpy() != 0
    f64 = np.zeros(shots, bool)
    ndiff = 0
    for part, h, (bp, rows), syn, err, stab, tag in ((0, code.hz, bz, sx, ex, code.hx, "x"),
                                                      (1, code.hx, bx, sz, ez, code.hz, "z")):
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, alpha=wl.alpha)
        f64 |= oracle.failures(stab, words(err), ref.corr)
        ndiff += int((words(out[f"corr_{tag}"]) != ref.corr).any(axis=-1).sum())
    k, nshots = int(f64.sum()), shots
    z = 1.959964
    ph = k / nshots
    den = 1 + z * z / nshots
    mid = (ph + z * z / (2 * nshots)) / den
    half = z * np.sqrt(ph * (1 - ph) / nshots + z * z / (4 * nshots * nshots)) / den
    ler = float(fail.mean())
    say(f"  GPU LER {ler:.4f}, FP64 LER {ph:.4f} CI [{mid - half:.4f}, {mid + half:.4f}], "
        f"corrections differing in {ndiff} (shot, part) pairs")
    assert mid - half <= ler <= mid + half
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


@pytest.mark.parametrize("key,p,spread", [("bb144_L16_T50", 0.08, 240), ("bb288_L32_T100", 0.03, 112),
                                          ("qc882_L64_T100", 0.03, 48)])
def test_full_size_sampled_shots_bit_exact(pk, key, p, spread):
    """The workloads at full size through the persistent batched form with the
    default launch shape: [[144,12,12]] L = 16, T = 50, 10^6 shots at the heaviest
    error rate; [[288,12,18]] L = 32, T = 100, 10^7 shots; the n = 882 stand-in
    L = 64, T = 100, 10^6 shots at the heaviest rate.  Sampled shots (the first 8,
    the last 8 and some spread over the range) are recomputed one by one by the
    FP32 oracle from its own sampler: corrections, chosen representation,
    convergence masks and failure flags equal bit for bit."""
    wl = WORKLOADS[key]
    code = wl.code()
    shots, shot0 = wl.shots, 3 * wl.shots
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"full size {key} p={p} shots={shots} (sampled shots vs oracle)")
    ex, ez, sx, sz = dec.sample(wl.seed, p, shot0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode_batched(sx, sz, prior, prior)
    fail = dec.failures(ex, ez, out["corr_x"], out["corr_z"])
    torch.cuda.synchronize()
    rng = np.random.default_rng(8)
    pick = np.unique(np.concatenate([np.arange(8), np.arange(shots - 8, shots),
                                     rng.choice(shots, spread, replace=False)]))
    samp = [oracle.sample(code.hx, code.hz, wl.seed, p, shot0 + int(i), 1) for i in pick]
    oex, oez, osx, osz = (np.concatenate([t[k] for t in samp]) for k in range(4))
    np.testing.assert_array_equal(words(sx)[pick], osx)
    np.testing.assert_array_equal(words(sz)[pick], osz)
    fail_ref = np.zeros(len(pick), np.uint8)
    for part, h, (bp, rows), syn, err, stab in ((0, code.hz, bz, osx, oex, code.hx),
                                                 (1, code.hx, bx, osz, oez, code.hz)):
        ref = oracle.decode(h, bp, rows, syn, np.full(code.n, mu), wl.T, alpha=wl.alpha, precision="f32")
        tag = "x" if part == 0 else "z"
        np.testing.assert_array_equal(words(out[f"corr_{tag}"])[pick], ref.corr)
        np.testing.assert_array_equal(out[f"basis_{tag}"].cpu().numpy()[pick], ref.chosen)
        mask = (ref.conv.astype(np.uint64) << np.arange(wl.L, dtype=np.uint64)).sum(axis=1).astype(np.uint64)
        np.testing.assert_array_equal(words(out[f"conv_{tag}"])[pick], mask)
        fail_ref |= oracle.failures(stab, err, ref.corr).astype(np.uint8) << part
    np.testing.assert_array_equal(fail.cpu().numpy()[pick], fail_ref)
    say(f"  {len(pick)} sampled shots equal; LER over all {shots}: {float((fail.cpu().numpy() != 0).mean()):.3e}")
    dec.close()


def test_degenerate_inputs(pk):
    """Edge cases of the method and of the boundary: zero syndromes (p = 0: every
    representation converges at t = 0 to the all-zero decision, the least-weight
    rule picks representation 0), T = 0 (only the t = 0 halting test: bit-exact
    against the oracle, unconverged shots decide all-zero), a single shot, and
    rejected sizes (0 shots, more than max_batch, p = 0 for the whole path) that
    fail with MBBP_EINVAL before any launch."""
    wl = WORKLOADS["bb72_L4_T20"]
    code = wl.code()
    mu = f32(oracle.prior_llr(0.05))
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=64)
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    say("degenerate inputs: zero syndromes, one shot, rejected sizes")
    ex, ez, sx, sz = dec.sample(wl.seed, 0.0, 0, 64)
    cand, kstat, _ = dec.decode_detail(0, sx, prior)
    out = dec.decode_batched(sx, sz, prior, prior)
    torch.cuda.synchronize()
    assert not words(ex).any() and not words(sx).any() and not words(sz).any()
    assert (kstat.cpu().numpy().view(np.uint16) == 0x8000).all()   # converged at K = 0
    assert not words(cand).any()
    for tag in ("x", "z"):
        assert not words(out[f"corr_{tag}"]).any()
        assert (words(out[f"conv_{tag}"]) == (1 << wl.L) - 1).all()
        assert (out[f"basis_{tag}"].cpu().numpy() == 0).all()
    # one shot, bit-exact
    _, _, sx1, _ = dec.sample(wl.seed, 0.05, 12345, 1)
    cand1, kstat1, _ = dec.decode_detail(0, sx1, prior)
    torch.cuda.synchronize()
    _, _, osx1, _ = oracle.sample(code.hx, code.hz, wl.seed, 0.05, 12345, 1)
    ref1 = oracle.decode(code.hz, *bz, osx1, np.full(code.n, mu), wl.T, alpha=wl.alpha, precision="f32")
    np.testing.assert_array_equal(words(cand1), ref1.cand)
    np.testing.assert_array_equal(kstat1.cpu().numpy().view(np.uint16) & 0x7FFF, ref1.K)
    for call in (lambda: dec.sample(1, 0.05, 0, 0), lambda: dec.sample(1, 0.05, 0, 65),
                 lambda: dec.run(1, 0.05, 0, 65), lambda: dec.run(1, 0.0, 0, 10)):
        with pytest.raises(pk.MbbpError) as ei:
            call()
        assert ei.value.status == -1
    dec.close()
    # T = 0
    shots = 300
    dec0, bx, bz = make_decoder(pk, code, wl, T=0, max_batch=shots)
    _, _, sx, sz = dec0.sample(wl.seed, 0.05, 0, shots)
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        cand, kstat, llr = dec0.decode_detail(part, syn, prior, want_llr=True)
        out = dec0.decode(sx, sz, prior, prior)
        torch.cuda.synchronize()
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), 0, alpha=wl.alpha, want_llr=True,
                            precision="f32")
        ks = kstat.cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(ks & 0x7FFF, ref.K)
        np.testing.assert_array_equal((ks >> 15).astype(bool), ref.conv)
        np.testing.assert_array_equal(words(cand), ref.cand)
        np.testing.assert_array_equal(llr.cpu().numpy().view(np.uint32), ref.llr.astype(np.float32).view(np.uint32))
        tag = "x" if part == 0 else "z"
        np.testing.assert_array_equal(words(out[f"corr_{tag}"]), ref.corr)
        np.testing.assert_array_equal(out[f"basis_{tag}"].cpu().numpy(), ref.chosen)
    dec0.close()


@pytest.mark.parametrize("key,p,shots", [("bb144_L16_T50", 0.08, 3000), ("bb72_L4_T20", 0.1, 4000)])
def test_fws_decision_bit_exact(pk, key, p, shots):
    """The paper's FWS decision (Section III-B: frequency of a candidate in the list
    over its weight + 1) in the plain and batched paths: corrections, chosen
    representation and failure flags equal the FP32 oracle's, and FWS picks
    differently from least weight on some shots."""
    wl = WORKLOADS[key]
    code = wl.code()
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, select=pk.FWS)
    lw, _, _ = make_decoder(pk, code, wl, max_batch=shots)
    say(f"FWS decision {key} p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(wl.seed, p, 4242, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode(sx, sz, prior, prior)
    outb = dec.decode_batched(sx, sz, prior, prior)
    outl = lw.decode(sx, sz, prior, prior)
    fail = dec.failures(ex, ez, out["corr_x"], out["corr_z"])
    torch.cuda.synchronize()
    differ = 0
    fail_ref = np.zeros(shots, np.uint8)
    for part, h, (bp, rows), syn, err, stab in ((0, code.hz, bz, sx, ex, code.hx),
                                                 (1, code.hx, bx, sz, ez, code.hz)):
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, alpha=wl.alpha,
                            select_rule=oracle.FWS, precision="f32")
        tag = "x" if part == 0 else "z"
        for o in (out, outb):
            np.testing.assert_array_equal(words(o[f"corr_{tag}"]), ref.corr)
            np.testing.assert_array_equal(o[f"basis_{tag}"].cpu().numpy(), ref.chosen)
        differ += int((outl[f"basis_{tag}"].cpu().numpy() != ref.chosen).sum())
        fail_ref |= oracle.failures(stab, words(err), ref.corr).astype(np.uint8) << part
    np.testing.assert_array_equal(fail.cpu().numpy(), fail_ref)
    assert differ > 0
    say(f"  FWS and least weight choose differently on {differ} (shot, part) pairs")
    dec.close()
    lw.close()


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


def test_run_counters_match_oracle(pk):
    """mbbp_run (sample -> batched BP -> decision -> failure test -> counters) equals
    the FP32 oracle's failures, iteration sums, edge-update count and
    non-convergence count exactly."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p, shot0 = 1200, 0.08, 99
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"mbbp_run counters bb144 p={p} shots={shots}")
    _run_vs_oracle(pk, dec, code, wl, bx, bz, p, shot0, shots)
    dec.close()


def test_run_x_only_layered_matches_oracle(pk):
    """The paper's experimental conditions (Section IV): X errors only (binary
    symmetric channel, prior log((1 - p) / p)), layered schedule, T = 100; mbbp_run's
    counters equal the FP32 oracle's exactly (part Z sees no errors)."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p, shot0, T = 500, 0.07, 4321, 100
    dec, bx, bz = make_decoder(pk, code, wl, T=T, max_batch=shots, schedule=pk.LAYERED, select=pk.FWS)
    dec.set_noise(pk.X_ONLY)
    say(f"mbbp_run x-only layered FWS bb144 p={p} shots={shots} T={T}")
    cnt = _run_vs_oracle(pk, dec, code, wl, bx, bz, p, shot0, shots, T=T, schedule=oracle.LAYERED,
                         noise=oracle.BSC_X, select_rule=oracle.FWS)
    assert cnt[pk.CNT_FAIL_Z] == 0 and cnt[pk.CNT_FAIL] == cnt[pk.CNT_FAIL_X]
    dec.close()


def _run_vs_oracle(pk, dec, code, wl, bx, bz, p, shot0, shots, T=None, schedule=None, noise=None,
                   select_rule=None):
    T = wl.T if T is None else T
    schedule = oracle.FLOODING if schedule is None else schedule
    noise = oracle.DEPOLARIZING if noise is None else noise
    cnt = dec.run(wl.seed, p, shot0, shots).cpu().numpy()
    ex, ez, sx, sz = oracle.sample(code.hx, code.hz, wl.seed, p, shot0, shots, noise)
    mu = f32(oracle.prior_llr(p, noise))
    fails = np.zeros((2, shots), bool)
    kmax = np.zeros(shots, np.int64)
    sum_k = edges = noconv = 0
    for part, h, (bp, rows), syn, err, stab in ((0, code.hz, bz, sx, ex, code.hx), (1, code.hx, bx, sz, ez, code.hz)):
        ref = oracle.decode(h, bp, rows, syn, np.full(code.n, mu), T, schedule=schedule, alpha=wl.alpha,
                            select_rule=oracle.MIN_WEIGHT if select_rule is None else select_rule,
                            precision="f32")
        fails[part] = oracle.failures(stab, err, ref.corr)
        kmax = np.maximum(kmax, ref.K.max(axis=1))
        sum_k += int(ref.K.sum())
        E = h.sum() + np.array([h[rows[bp[l]:bp[l + 1]]].sum() for l in range(wl.L)])
        edges += int((ref.K * E[None, :]).sum())
        noconv += int((ref.chosen < 0).sum())
    expect = {pk.CNT_FAIL: int((fails[0] | fails[1]).sum()), pk.CNT_FAIL_X: int(fails[0].sum()),
              pk.CNT_FAIL_Z: int(fails[1].sum()), pk.CNT_SUM_KMAX: int(kmax.sum()), pk.CNT_SUM_K: sum_k,
              pk.CNT_EDGE_UPDATES: edges, pk.CNT_NOCONV: noconv}
    for k, v in expect.items():
        assert int(cnt[k]) == v, (k, int(cnt[k]), v)
    say(f"  counters {cnt.tolist()}")
    return cnt


@pytest.mark.parametrize("factory", [codes.steane7, codes.surface13, codes.toric18])
def test_nms_small_codes_padded_rows_bit_exact(pk, factory):
    """Rows of weight 2..4 (padded row slots) and variables of degree 1..4 (masked
    variable passes): bit-exact against the FP32 oracle."""
    from workloads.perms import check_permutations
    code = factory()
    L, T, shots, p = 3, 12, 700, 0.1
    bx = oracle.build_bases(code.hx, "ramp", L, check_permutations(code.hx.shape[0], L, 1))
    bz = oracle.build_bases(code.hz, "ramp", L, check_permutations(code.hz.shape[0], L, 1))
    say(f"small code {code.name}: n={code.n}")
    dec = pk.Decoder(code.hx, code.hz, bx, bz, T, alpha=0.8, max_batch=shots)
    ex, ez, sx, sz = dec.sample(5, p, 0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
        torch.cuda.synchronize()
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), T, alpha=0.8, want_llr=True,
                            precision="f32")
        ks = kstat.cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(words(cand), ref.cand)
        np.testing.assert_array_equal(ks & 0x7FFF, ref.K)
        np.testing.assert_array_equal(llr.cpu().numpy().view(np.uint32), ref.llr.astype(np.float32).view(np.uint32))
    dec.close()


@pytest.mark.parametrize("key,p", [("bb144_L16_T50", 0.07), ("bb72_L4_T20", 0.06)])
def test_launch_configs_bit_identical(pk, key, p):
    """Every launch shape (lanes per instance, waves per block, shots per item, plain
    or persistent) gives the same bits; the reference is the FP32 oracle."""
    wl = WORKLOADS[key]
    code = wl.code()
    shots = 999
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    ex, ez, sx, sz = dec.sample(11, p, 3, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    ref = {}
    for part, h, (bp, rows), syn, tag in ((0, code.hz, bz, sx, "x"), (1, code.hx, bx, sz, "z")):
        r = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, alpha=wl.alpha, precision="f32")
        ref[tag] = r
    for lpi in (64,):
        for wpb, chunk in ((1, 1), (4, 7), (2, 64), (3, 1000)):
            for form in (0, 1):
                try:
                    dec.set_config(form, lpi, wpb, chunk, 37 if form else 0)
                except pk.MbbpError as e:
                    assert e.status == -5
                    continue
                say(f"  {key} lpi={lpi} wpb={wpb} chunk={chunk} form={form}")
                out = (dec.decode if form == 0 else dec.decode_batched)(sx, sz, prior, prior)
                torch.cuda.synchronize()
                for tag in ("x", "z"):
                    np.testing.assert_array_equal(words(out[f"corr_{tag}"]), ref[tag].corr)
                    np.testing.assert_array_equal(out[f"basis_{tag}"].cpu().numpy(), ref[tag].chosen)
    dec.close()


SERIAL_KERNELS = ("SERIAL_SLOTS", "SERIAL_LANES", "SERIAL_LEVELS")


@pytest.mark.parametrize("key,p,shots", [("bb72_L4_T20", 0.05, 3000), ("bb144_L16_T50", 0.06, 500)])
def test_nms_serial_bit_exact_fp32(pk, key, p, shots):
    """Serial schedule: each of the three serial kernels (eight lanes per shot, one
    shot per lane, level-synchronous) equals the oracle's row-order sweep bit for bit
    (decisions, iterations, convergence, posterior bits); the eight-lane kernel also
    without posteriors (its other instantiation)."""
    wl = WORKLOADS[key]
    code = wl.code()
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, schedule=pk.LAYERED)
    say(f"nms serial fp32 bit-exact {key} p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(wl.seed, p, 0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, schedule=oracle.LAYERED,
                            alpha=wl.alpha, want_llr=True, precision="f32")
        for kern in SERIAL_KERNELS:
            say(f"  part {part} kernel {kern}")
            dec.set_serial_kernel(getattr(pk, kern))
            cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
            torch.cuda.synchronize()
            ks = kstat.cpu().numpy().view(np.uint16)
            np.testing.assert_array_equal(ks & 0x7FFF, ref.K)
            np.testing.assert_array_equal((ks >> 15).astype(bool), ref.conv)
            np.testing.assert_array_equal(words(cand), ref.cand)
            np.testing.assert_array_equal(llr.cpu().numpy().view(np.uint32),
                                          ref.llr.astype(np.float32).view(np.uint32))
        dec.set_serial_kernel(pk.SERIAL_SLOTS)
        cand, kstat, _ = dec.decode_detail(part, syn, prior, want_llr=False)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(kstat.cpu().numpy().view(np.uint16) & 0x7FFF, ref.K)
        np.testing.assert_array_equal(words(cand), ref.cand)
        say(f"  part {part}: mean K {ref.K.mean():.3f}")
    dec.close()


@pytest.mark.parametrize("factory", [codes.steane7, codes.surface13, codes.toric18])
def test_nms_serial_small_codes_bit_exact(pk, factory):
    from workloads.perms import check_permutations
    code = factory()
    L, T, shots, p = 3, 12, 500, 0.1
    bx = oracle.build_bases(code.hx, "ramp", L, check_permutations(code.hx.shape[0], L, 1))
    bz = oracle.build_bases(code.hz, "ramp", L, check_permutations(code.hz.shape[0], L, 1))
    say(f"serial small code {code.name}")
    dec = pk.Decoder(code.hx, code.hz, bx, bz, T, alpha=0.8, max_batch=shots, schedule=pk.LAYERED)
    ex, ez, sx, sz = dec.sample(5, p, 0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), T, schedule=oracle.LAYERED, alpha=0.8,
                            want_llr=True, precision="f32")
        for kern in SERIAL_KERNELS:
            dec.set_serial_kernel(getattr(pk, kern))
            cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(words(cand), ref.cand)
            np.testing.assert_array_equal(kstat.cpu().numpy().view(np.uint16) & 0x7FFF, ref.K)
            np.testing.assert_array_equal(llr.cpu().numpy().view(np.uint32),
                                          ref.llr.astype(np.float32).view(np.uint32))
    dec.close()


def test_spa_serial_exact_on_trees(pk):
    """Serial sum-product on cycle-free graphs reaches the exact marginals (FP64 oracle)."""
    from .test_oracle_pins import _random_tree
    rng = np.random.default_rng(22)
    bases = (np.zeros(2, np.int32), np.zeros(0, np.int32))
    for trial in range(4):
        h = _random_tree(rng, int(rng.integers(3, 7)), wmin=3, wmax=5)
        n = h.shape[1]
        say(f"spa serial tree trial {trial} n={n}")
        dec = pk.Decoder(h, _commuting_pair(h), bases, bases, 30, rule=pk.SPA, fixed_T=True, max_batch=64,
                         schedule=pk.LAYERED)
        s = rng.integers(0, 2, (64, h.shape[0])).astype(np.uint8)
        syn = torch.from_numpy(oracle.pack(s).view(np.int64)).cuda()
        mu = rng.uniform(-1.0, 3.0, n).astype(np.float32)
        cand, kstat, llr = dec.decode_detail(1, syn, torch.from_numpy(mu).cuda(), want_llr=True)
        torch.cuda.synchronize()
        ref = oracle.decode(h, np.array([0, 0], np.int32), np.array([], np.int32), oracle.pack(s),
                            mu.astype(np.float64), 30, schedule=oracle.LAYERED, rule=oracle.SPA, fixed_T=True,
                            want_llr=True)
        got = llr.cpu().numpy()[:, 0, :].astype(np.float64)
        exp = ref.llr[:, 0, :]
        err = np.abs(got - exp) / np.maximum(1.0, np.abs(exp))
        say(f"  max relative LLR error {err.max():.3e}")
        assert np.all(err <= 1e-4)
        dec.close()


def test_run_graph_replays_equal_direct_launches(pk):
    """mbbp_run replays one captured graph per batch size; every replay (with eager work
    and synchronisations in between) gives the counters of direct launches."""
    wl = WORKLOADS["bb72_L4_T20"]
    code = wl.code()
    shots = 3000
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    calls = [(1, 0.05, 0), (2, 0.08, 123), (3, 0.03, 10**7), (1, 0.05, 0)]
    direct = []
    dec.set_graph(False)
    for seed, p, shot0 in calls:
        direct.append(dec.run(seed, p, shot0, shots).cpu().numpy())
    dec.set_graph(True)
    for rep in range(2):
        for (seed, p, shot0), ref in zip(calls, direct):
            say(f"graph replay {rep} seed={seed} p={p} shot0={shot0}")
            junk = torch.randn(1000, device="cuda").sum()   # eager work between replays
            got = dec.run(seed, p, shot0, shots).cpu().numpy()
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got, ref)
            assert float(junk) == float(junk)
    # accumulation into the caller's counters
    acc = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
    dec.run(1, 0.05, 0, shots, acc)
    dec.run(2, 0.08, 123, shots, acc)
    np.testing.assert_array_equal(acc.cpu().numpy(), direct[0] + direct[1])
    dec.close()


def test_autotune_keeps_results(pk):
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots = 4000
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    ex, ez, sx, sz = dec.sample(5, 0.06, 0, shots)
    prior = torch.full((code.n,), f32(oracle.prior_llr(0.06)), dtype=torch.float32, device="cuda")
    before = dec.decode_batched(sx, sz, prior, prior)
    b0 = {k: v.cpu().numpy() for k, v in before.items()}
    for form in (0, 1):
        cfg = dec.autotune(form, seed=9, p=0.05, shots=shots)
        say(f"autotune form {form}: {cfg}")
        assert cfg == dec.get_config(form)
    after = dec.decode_batched(sx, sz, prior, prior)
    plain = dec.decode(sx, sz, prior, prior)
    torch.cuda.synchronize()
    for k in b0:
        np.testing.assert_array_equal(after[k].cpu().numpy(), b0[k], err_msg=k)
        np.testing.assert_array_equal(plain[k].cpu().numpy(), b0[k], err_msg=k)
    dec.close()


@pytest.mark.parametrize("factory,L,T,p,shots", [(codes.bb288, 6, 40, 0.04, 80), (codes.qc882, 6, 30, 0.02, 40)])
def test_nms_large_codes_bit_exact(pk, factory, L, T, p, shots):
    """Codes whose representations need 5 or 14 passes of 64 lanes (the latter in the
    compact LDS layout, one byte per decision): bit-exact against the FP32 oracle."""
    from workloads.perms import check_permutations
    code = factory()
    bx = oracle.build_bases(code.hx, "ramp", L, check_permutations(code.hx.shape[0], L, 3))
    bz = oracle.build_bases(code.hz, "ramp", L, check_permutations(code.hz.shape[0], L, 3))
    say(f"large code {code.name}: n={code.n} L={L} T={T} shots={shots}")
    dec = pk.Decoder(code.hx, code.hz, bx, bz, T, alpha=0.875, max_batch=shots)
    ex, ez, sx, sz = dec.sample(11, p, 0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
        torch.cuda.synchronize()
        ref = oracle.decode(h, bp, rows, words(syn), np.full(code.n, mu), T, alpha=0.875, want_llr=True,
                            precision="f32")
        ks = kstat.cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(words(cand), ref.cand)
        np.testing.assert_array_equal(ks & 0x7FFF, ref.K)
        np.testing.assert_array_equal(llr.cpu().numpy().view(np.uint32), ref.llr.astype(np.float32).view(np.uint32))
        say(f"  part {part}: mean K {ref.K.mean():.2f}")
    dec.close()


@pytest.mark.parametrize("key,p,shots", [("bb144_L16_T50", 0.08, 2001), ("bb72_L4_T20", 0.06, 3001)])
def test_paired_instances_equal_one_per_wave(pk, key, p, shots):
    """Two instances per wavefront (default for flooding min-sum) and one instance per
    wavefront give the same bits: per-representation decisions, iteration counts,
    convergence flags and posteriors, in the plain and the persistent form, with work
    items of an odd number of shots (one instance of a wave idles at the end)."""
    wl = WORKLOADS[key]
    code = wl.code()
    decs = [make_decoder(pk, code, wl, max_batch=shots, one_per_wave=one)[0] for one in (False, True)]
    ex, ez, sx, sz = decs[0].sample(5, p, 7, shots)
    prior = torch.full((code.n,), f32(oracle.prior_llr(p)), dtype=torch.float32, device="cuda")
    say(f"paired vs one per wave {key} p={p} shots={shots}")
    for part, syn in ((0, sx), (1, sz)):
        got = []
        for d in decs:
            cand, kstat, llr = d.decode_detail(part, syn, prior, want_llr=True)
            torch.cuda.synchronize()
            got.append((words(cand), kstat.cpu().numpy(), llr.cpu().numpy().view(np.uint32)))
        for a, b, what in zip(got[0], got[1], ("decisions", "iterations", "posterior bits")):
            np.testing.assert_array_equal(a, b, err_msg=f"part {part} {what}")
    for chunk in (1, 7, 64):
        outs = []
        for d in decs:
            d.set_config(1, 64, 4, chunk, 64)
            outs.append(d.decode_batched(sx, sz, prior, prior))
        torch.cuda.synchronize()
        for k in outs[0]:
            np.testing.assert_array_equal(outs[0][k].cpu().numpy(), outs[1][k].cpu().numpy(),
                                          err_msg=f"chunk {chunk} {k}")
    for d in decs:
        d.close()
