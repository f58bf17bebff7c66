"""GPU parity of the cases the first parity suite leaves out, through the C ABI:

* sum-product on codes with cycles ([[72]], [[144]], both schedules) against the
  FP64 oracle: every posterior within 1e-4 * max(1, |LLR|) after a short fixed
  horizon, decisions equal except on tie-prone instances (counted);
* the serial schedule on the five-pass [[288]] and fourteen-pass n = 882 kernels,
  bit-exact against the FP32 oracle;
* per-shot priors through mbbp_decode and mbbp_decode_batched, both parts;
* the paper's Table II inputs (tree and matched random augmentation) through
  mbbp_decode;
* the tie counter of mbbp_run under both decision rules;
* the full-horizon comparison with the FP64 oracle, paired shot by shot;
* mbbp_run's graph re-captured after the launch shape changes, and graph
  replays timed by the graph's own event nodes.
"""

import concurrent.futures
import math
import sys

import numpy as np
import pytest

import oracle
from workloads import codes
from workloads.configs import WORKLOADS
from workloads.partitions import matched_random_bases, tree_bases
from workloads.perms import check_permutations

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


def words(t):
    return t.detach().cpu().numpy().view(np.uint64)


def make_decoder(pk, code, wl, T=None, **kw):
    bx = bases_for(code.hx, wl, oracle.build_bases)
    bz = bases_for(code.hz, wl, oracle.build_bases)
    dec = pk.Decoder(code.hx, code.hz, bx, bz, wl.T if T is None else T, alpha=kw.pop("alpha", wl.alpha), **kw)
    return dec, bx, bz


def oracle_decode_par(h, bp, rows, syn, prior, T, threads=16, chunk=512, **kw):
    """The oracle over disjoint shot ranges on host threads (each call is the plain
    single-threaded oracle); results concatenated in shot order."""
    shots = syn.shape[0]
    ranges = [(a, min(a + chunk, shots)) for a in range(0, shots, chunk)]

    def one(r):
        pr = prior[r[0]:r[1]] if prior.ndim == 2 else prior
        return oracle.decode(h, bp, rows, syn[r[0]:r[1]], pr, T, **kw)

    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, ranges))
    cat = lambda f: None if getattr(res[0], f) is None else np.concatenate([getattr(r, f) for r in res])  # noqa
    return oracle.DecodeResult(cat("cand"), cat("K"), cat("conv"), cat("llr"), cat("margin"), cat("clamp"),
                               cat("chosen"), cat("corr"))


def mcnemar_p(b, c):
    """Two-sided exact McNemar p-value for b, c discordant pairs."""
    n = b + c
    if n == 0:
        return 1.0
    k = min(b, c)
    tail = sum(math.comb(n, i) for i in range(k + 1)) / 2.0 ** n
    return min(1.0, 2.0 * tail)


# ------------------------------------------------------------------ sum-product on codes with cycles

@pytest.mark.parametrize("key,p,shots", [("bb72_L4_T20", 0.05, 2000), ("bb144_L16_T50", 0.06, 600)])
@pytest.mark.parametrize("rule,schedule", [(1, 0), (1, 1), (0, 1)])
def test_short_horizon_fp64(pk, key, p, shots, rule, schedule):
    """Sum-product (Section II-B's product-sum rule) and serial min-sum on the codes'
    representations, fixed horizon T = 5, against the FP64 oracle: hard decisions,
    iteration counts and convergence equal except on tie-prone instances (FP64
    margin < 1e-3, counted); posteriors within 1e-4 * max(1, |LLR|).  In the serial
    schedule messages grow to hundreds within the horizon and a posterior of order 1
    is a sum of such terms, so single-precision rounding is relative to the
    instance's largest posterior: there the bound is 1e-4 * max(1, max_j |LLR_j| of
    the instance), and the entries beyond the per-entry bound are counted, together
    with those of the single-precision oracle (a different evaluation of the same
    rule) as a reference for what FP32 gives."""
    wl = WORKLOADS[key]
    code = wl.code()
    dec, bx, bz = make_decoder(pk, code, wl, T=5, max_batch=shots, rule=rule, fixed_T=True, schedule=schedule)
    say(f"{('NMS', 'SPA')[rule]} {key} schedule={schedule} p={p} shots={shots} T=5 vs FP64")
    ex, ez, sx, sz = dec.sample(wl.seed, p, 321, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
        torch.cuda.synchronize()
        kw = dict(schedule=schedule, rule=rule, alpha=wl.alpha, fixed_T=True, want_llr=True)
        ref = oracle_decode_par(h, bp, rows, words(syn), np.full(code.n, mu), 5, **kw)
        ref32 = oracle_decode_par(h, bp, rows, words(syn), np.full(code.n, mu), 5, precision="f32", **kw)
        ks = kstat.cpu().numpy().view(np.uint16)
        K, conv = (ks & 0x7FFF).astype(np.int32), (ks >> 15).astype(bool)
        same = (words(cand) == ref.cand).all(axis=-1) & (K == ref.K) & (conv == ref.conv)
        tie = tie_shots(ref.margin)
        got = llr.cpu().numpy().astype(np.float64)
        err = np.abs(got - ref.llr) / np.maximum(1.0, np.abs(ref.llr))
        err32 = np.abs(ref32.llr - ref.llr) / np.maximum(1.0, np.abs(ref.llr))
        scale = np.maximum(1.0, np.abs(ref.llr).max(axis=-1, keepdims=True))
        err_inst = np.abs(got - ref.llr) / scale
        say(f"  part {part}: differing instances {int((~same).sum())} of {same.size} (tie-prone {int(tie.sum())}); "
            f"max relative LLR error {err.max():.2e} ({int((err > 1e-4).sum())} entries beyond 1e-4; "
            f"single-precision oracle {err32.max():.2e}, {int((err32 > 1e-4).sum())} entries), "
            f"relative to the instance's largest posterior {err_inst.max():.2e}")
        assert not (~same & ~tie).any(), "decision differs from FP64 on a non-tie instance"
        if schedule == 0:
            assert err.max() <= 1e-4
        else:
            assert err_inst.max() <= 1e-4
    dec.close()


def test_spa_full_horizon_paired_fp64(pk):
    """Sum-product decoding with early stop at T = 50 on [[144]]: failures paired shot
    by shot with the FP64 oracle's (exact McNemar test of equal failure rates), and
    corrections equal on all but a few per cent of (shot, part) pairs."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p = 4000, 0.05
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, rule=pk.SPA)
    say(f"spa full horizon bb144 p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(wl.seed, p, 777, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode(sx, sz, prior, prior)
    fail = dec.failures(ex, ez, out["corr_x"], out["corr_z"]).cpu().numpy() != 0
    f64 = np.zeros(shots, bool)
    ndiff = 0
    for h, (bp, rows), syn, err, stab, tag in ((code.hz, bz, sx, ex, code.hx, "x"),
                                                (code.hx, bx, sz, ez, code.hz, "z")):
        ref = oracle_decode_par(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, rule=oracle.SPA)
        f64 |= oracle.failures(stab, words(err), ref.corr)
        ndiff += int((words(out[f"corr_{tag}"]) != ref.corr).any(axis=-1).sum())
    b, c = int((fail & ~f64).sum()), int((~fail & f64).sum())
    pv = mcnemar_p(b, c)
    say(f"  GPU LER {fail.mean():.4e}, FP64 LER {f64.mean():.4e}, discordant {b}/{c} (McNemar p {pv:.3f}), "
        f"corrections differing in {ndiff} of {2 * shots} (shot, part) pairs")
    assert pv > 1e-3
    assert ndiff <= 0.05 * 2 * shots
    dec.close()


# ------------------------------------------------------------------ serial schedule on the large codes

@pytest.mark.parametrize("factory,L,T,p,shots", [(codes.bb288, 6, 40, 0.04, 80), (codes.qc882, 6, 30, 0.02, 40)])
def test_nms_serial_large_codes_bit_exact(pk, factory, L, T, p, shots):
    """Serial schedule on representations of 5 and 14 check passes (the n = 882
    code in the compact LDS layout): bit-exact against the FP32 oracle's row-order
    sweep (decisions, iterations, posterior bits)."""
    code = factory()
    bx = oracle.build_bases(code.hx, "ramp", L, check_permutations(code.hx.shape[0], L, 3))
    bz = oracle.build_bases(code.hz, "ramp", L, check_permutations(code.hz.shape[0], L, 3))
    say(f"serial large code {code.name}: n={code.n} L={L} T={T} shots={shots}")
    dec = pk.Decoder(code.hx, code.hz, bx, bz, T, alpha=0.875, max_batch=shots, schedule=pk.LAYERED)
    ex, ez, sx, sz = dec.sample(11, p, 0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        ref = oracle_decode_par(h, bp, rows, words(syn), np.full(code.n, mu), T, schedule=oracle.LAYERED,
                                alpha=0.875, want_llr=True, precision="f32", chunk=8)
        for kern in (pk.SERIAL_SLOTS, pk.SERIAL_LANES):
            say(f"  part {part} serial kernel {kern}")
            dec.set_serial_kernel(kern)
            cand, kstat, llr = dec.decode_detail(part, syn, prior, want_llr=True)
            torch.cuda.synchronize()
            ks = kstat.cpu().numpy().view(np.uint16)
            np.testing.assert_array_equal(words(cand), ref.cand)
            np.testing.assert_array_equal(ks & 0x7FFF, ref.K)
            np.testing.assert_array_equal((ks >> 15).astype(bool), ref.conv)
            np.testing.assert_array_equal(llr.cpu().numpy().view(np.uint32),
                                          ref.llr.astype(np.float32).view(np.uint32))
        say(f"  part {part}: mean K {ref.K.mean():.2f}")
    dec.close()


# ------------------------------------------------------------------ per-shot priors through the decoders

@pytest.mark.parametrize("schedule", [0, 1])
def test_per_shot_priors_decode_and_batched(pk, schedule):
    """prior_per_shot = 1 through mbbp_decode and mbbp_decode_batched, both parts:
    corrections, chosen representation and convergence masks equal the FP32
    oracle's on non-uniform soft priors (some negative)."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots = 1200
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, schedule=schedule)
    say(f"per-shot priors decode/decode_batched bb144 schedule={schedule} shots={shots}")
    ex, ez, sx, sz = dec.sample(17, 0.05, 50, shots)
    rng = np.random.default_rng(12)
    prx = rng.uniform(-0.5, 5.0, (shots, code.n)).astype(np.float32)
    prz = rng.uniform(0.5, 6.0, (shots, code.n)).astype(np.float32)
    tx, tz = torch.from_numpy(prx).cuda(), torch.from_numpy(prz).cuda()
    outs = [dec.decode(sx, sz, tx, tz), dec.decode_batched(sx, sz, tx, tz)]
    if schedule == 1:  # the serial schedule's one-shot-per-lane kernel too
        dec.set_serial_kernel(pk.SERIAL_LANES)
        outs += [dec.decode(sx, sz, tx, tz), dec.decode_batched(sx, sz, tx, tz)]
    torch.cuda.synchronize()
    for h, (bp, rows), syn, pr, tag in ((code.hz, bz, sx, prx, "x"), (code.hx, bx, sz, prz, "z")):
        ref = oracle_decode_par(h, bp, rows, words(syn), pr.astype(np.float64), wl.T, schedule=schedule,
                                alpha=wl.alpha, precision="f32")
        mask = (ref.conv.astype(np.uint64) << np.arange(wl.L, dtype=np.uint64)).sum(axis=1).astype(np.uint64)
        for o in outs:
            np.testing.assert_array_equal(words(o[f"corr_{tag}"]), ref.corr)
            np.testing.assert_array_equal(o[f"basis_{tag}"].cpu().numpy(), ref.chosen)
            np.testing.assert_array_equal(words(o[f"conv_{tag}"]), mask)
        say(f"  part {tag}: converged instances {ref.conv.mean():.3f}")
    dec.close()


# ------------------------------------------------------------------ Table II inputs

@pytest.mark.parametrize("mode", ["tree", "random"])
def test_partition_bases_decode_bit_exact(pk, mode):
    """The representations of one partition (Algorithm 2 on root order pi_2), as its
    subtrees or as matched random rows (Table II), decoded under the paper's
    conditions (layered schedule, FWS): equal to the FP32 oracle."""
    code = codes.bb144()
    perms_x = check_permutations(code.hx.shape[0], 3, seed=0)
    perms_z = check_permutations(code.hz.shape[0], 3, seed=0)
    sz_ = oracle.subtree_lists(code.hz, perms_z[2])
    sx_ = oracle.subtree_lists(code.hx, perms_x[2])
    L = len(sz_)
    if mode == "tree":
        bz, bx = tree_bases(sz_), tree_bases(sx_, count=L)
    else:
        bz = matched_random_bases(sz_, code.hz.shape[0], seed=0, k=2)
        bx = matched_random_bases(sx_, code.hx.shape[0], seed=0, k=2, count=L)
    shots, p, T = 1500, 0.06, 100
    say(f"partition bases {mode}: L={L}")
    dec = pk.Decoder(code.hx, code.hz, bx, bz, T, schedule=pk.LAYERED, alpha=0.875, select=pk.FWS,
                     max_batch=shots)
    dec.set_noise(pk.X_ONLY)
    ex, ez, sx, sz = dec.sample(3, p, 0, shots)
    mu = f32(oracle.prior_llr(p, oracle.BSC_X))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode(sx, sz, prior, prior)
    torch.cuda.synchronize()
    for h, (bp, rows), syn, tag in ((code.hz, bz, sx, "x"), (code.hx, bx, sz, "z")):
        ref = oracle_decode_par(h, bp, rows, words(syn), np.full(code.n, mu), T, schedule=oracle.LAYERED,
                                alpha=0.875, select_rule=oracle.FWS, precision="f32")
        np.testing.assert_array_equal(words(out[f"corr_{tag}"]), ref.corr)
        np.testing.assert_array_equal(out[f"basis_{tag}"].cpu().numpy(), ref.chosen)
    dec.close()


# ------------------------------------------------------------------ tie counter

def _ties(ref, W, rule):
    """(shot) count of decisions whose best value is shared by a distinct converged
    candidate, computed from the oracle's per-representation lists."""
    shots, L = ref.conv.shape
    wt = np.array([[sum(bin(int(x)).count("1") for x in ref.cand[s, l]) for l in range(L)] for s in range(shots)])
    n = 0
    for s in range(shots):
        b = int(ref.chosen[s])
        if b < 0:
            continue
        cands = [tuple(ref.cand[s, l]) for l in range(L)]
        if rule == oracle.MIN_WEIGHT:
            n += any(ref.conv[s, l] and wt[s, l] == wt[s, b] and cands[l] != cands[b] for l in range(L))
        else:
            conv = [l for l in range(L) if ref.conv[s, l]]
            cnt = {}
            for l in conv:
                cnt[cands[l]] = cnt.get(cands[l], 0) + 1
            best = (cnt[cands[b]], wt[s, b] + 1)
            n += any(c != cands[b] and cnt[c] * best[1] == best[0] * (sum(bin(int(x)).count("1") for x in c) + 1)
                     for c in cnt)
    return n


@pytest.mark.parametrize("select", [0, 1])
def test_run_tie_counter(pk, select):
    """MBBP_CNT_TIES of mbbp_run equals the count recomputed from the FP32 oracle's
    lists, under least weight and under FWS."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots, p, shot0 = 2000, 0.08, 31
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, select=select)
    say(f"tie counter select={select} bb144 p={p} shots={shots}")
    cnt = dec.run(wl.seed, p, shot0, shots).cpu().numpy()
    ex, ez, sx, sz = oracle.sample(code.hx, code.hz, wl.seed, p, shot0, shots)
    mu = f32(oracle.prior_llr(p))
    ties = 0
    for h, (bp, rows), syn in ((code.hz, bz, sx), (code.hx, bx, sz)):
        ref = oracle_decode_par(h, bp, rows, syn, np.full(code.n, mu), wl.T, alpha=wl.alpha, select_rule=select,
                                precision="f32")
        ties += _ties(ref, code.n, select)
    say(f"  ties {int(cnt[pk.CNT_TIES])} (oracle lists: {ties})")
    assert ties > 0
    assert int(cnt[pk.CNT_TIES]) == ties
    dec.close()


# ------------------------------------------------------------------ full horizon against FP64, paired

@pytest.mark.parametrize("key,p,shots,shot0", [("bb144_L16_T50", 0.06, 30000, 40000),
                                               ("bb72_L4_T20", 0.05, 10000, 0)])
def test_full_horizon_fp64_paired(pk, key, p, shots, shot0):
    """Full horizon with early stop against the FP64 oracle on the same shots.  At
    T = 20..50 single- and double-precision BP trajectories separate on about 1-3%
    of instances (the kernel equals the single-precision oracle bit for bit, so this
    is a property of FP32 BP).  Checked: (i) failures paired shot by shot, exact
    McNemar test of equal failure rates (p > 1e-3); (ii) per instance of part X,
    decisions, iterations and convergence differ only on instances whose FP64 run
    came within 3e-2 of a sign flip, and those beyond the 1e-3 tie margin are at
    most 2% of instances.  The counts are printed."""
    wl = WORKLOADS[key]
    code = wl.code()
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say(f"full-horizon FP64 paired {key} p={p} shots={shots}")
    ex, ez, sx, sz = dec.sample(wl.seed, p, shot0, shots)
    mu = f32(oracle.prior_llr(p))
    prior = torch.full((code.n,), mu, dtype=torch.float32, device="cuda")
    out = dec.decode(sx, sz, prior, prior)
    fail = dec.failures(ex, ez, out["corr_x"], out["corr_z"]).cpu().numpy() != 0
    cand, kstat, _ = dec.decode_detail(0, sx, prior)
    torch.cuda.synchronize()
    f64 = np.zeros(shots, bool)
    refs = []
    for h, (bp, rows), syn, err, stab in ((code.hz, bz, sx, ex, code.hx), (code.hx, bx, sz, ez, code.hz)):
        ref = oracle_decode_par(h, bp, rows, words(syn), np.full(code.n, mu), wl.T, alpha=wl.alpha)
        f64 |= oracle.failures(stab, words(err), ref.corr)
        refs.append(ref)
    b, c = int((fail & ~f64).sum()), int((~fail & f64).sum())
    pv = mcnemar_p(b, c)
    ref = refs[0]
    ks = kstat.cpu().numpy().view(np.uint16)
    same = (words(cand) == ref.cand).all(axis=-1) & ((ks & 0x7FFF) == ref.K) & ((ks >> 15).astype(bool) == ref.conv)
    mm = np.minimum(ref.margin[..., 0], ref.margin[..., 1])
    diff = ~same
    say(f"  GPU LER {fail.mean():.4e}, FP64 LER {f64.mean():.4e}; discordant shots {b} (GPU fails) / {c} "
        f"(FP64 fails), McNemar p {pv:.3f}")
    say(f"  part X instances {same.size}: differing {int(diff.sum())}: FP64 margin < 1e-3: "
        f"{int((diff & (mm < 1e-3)).sum())}, 1e-3..1e-2: {int((diff & (mm >= 1e-3) & (mm < 1e-2)).sum())}, "
        f">= 1e-2: {int((diff & (mm >= 1e-2)).sum())}; max margin of a differing instance "
        f"{(mm[diff].max() if diff.any() else 0.0):.3e}")
    assert pv > 1e-3
    assert not (diff & (mm >= 3e-2)).any()
    assert int((diff & (mm >= 1e-3)).sum()) <= 0.02 * same.size
    dec.close()


# ------------------------------------------------------------------ graph capture and timing

def test_graph_recaptured_after_config_change(pk):
    """mbbp_run's captured graph holds the batched launch shape; after mbbp_set_config
    and mbbp_autotune the next run replays a graph whose BP kernel node has the new
    shape, with unchanged counters."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots = 4000
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say("graph re-capture after config changes")
    c0 = dec.run(1, 0.06, 0, shots).cpu().numpy()
    g0 = dec.run_graph_config(shots)
    assert g0["blocks"] == dec.get_config(1)["blocks"] and g0["waves_per_block"] == dec.get_config(1)["waves_per_block"]
    dec.set_config(1, 64, 2, 16, 300)
    c1 = dec.run(1, 0.06, 0, shots).cpu().numpy()
    g1 = dec.run_graph_config(shots)
    assert g1["blocks"] == 300 and g1["waves_per_block"] == 2 and g1["chunk"] == 16, g1
    cfg = dec.autotune(1, seed=2, p=0.06, shots=shots)
    c2 = dec.run(1, 0.06, 0, shots).cpu().numpy()
    g2 = dec.run_graph_config(shots)
    assert (g2["blocks"], g2["waves_per_block"], g2["chunk"]) == (cfg["blocks"], cfg["waves_per_block"], cfg["chunk"])
    np.testing.assert_array_equal(c0, c1)
    np.testing.assert_array_equal(c0, c2)
    dec.close()


def test_graph_replay_timing(pk):
    """BP timing through graph replays (event record nodes given fresh events per
    replay) agrees with timing of direct launches within 20%, and the counters of
    timed and untimed replays are equal."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots = 100000
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    say("graph replay timing")
    ref = dec.run(1, 0.06, 0, shots).cpu().numpy()
    res = {}
    for graph in (True, False):
        dec.set_graph(graph)
        dec.bp_time(reset=True)
        dec.set_timing(True)
        got = [dec.run(1, 0.06, 0, shots).cpu().numpy() for _ in range(3)]
        dec.set_timing(False)
        ms, n = dec.bp_time(reset=True)
        assert n == 3
        for g in got:
            np.testing.assert_array_equal(g, ref)
        res[graph] = ms / n
    say(f"  BP per launch: graph replay {res[True]:.3f} ms, direct {res[False]:.3f} ms")
    assert 0.8 <= res[True] / res[False] <= 1.25
    dec.close()


# ------------------------------------------------------------------ plain form beyond the grid cap

@pytest.mark.parametrize("case", ["paired", "shared", "serial"])
def test_plain_grid_stride_equals_batched(pk, case):
    """The plain form launches one workgroup per work item up to a cap of 65536 and
    strides over the rest (the dispatch's thread count must fit 32 bits): with one
    shot per work item and more items than the cap, its corrections, chosen
    representations and convergence masks equal the persistent form's.  Cases: the
    paired kernel ([[72]]), the instance shared by seven wavefronts (n = 882), the
    serial kernel with eight lanes per shot ([[144]])."""
    if case == "paired":
        wl = WORKLOADS["bb72_L4_T20"]
        code, p, shots, sched = wl.code(), 0.05, 40000, 0
        dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    elif case == "shared":
        code, p, shots, sched, L = codes.qc882(), 0.02, 12000, 0, 6
        bx = oracle.build_bases(code.hx, "ramp", L, check_permutations(code.hx.shape[0], L, 3))
        bz = oracle.build_bases(code.hz, "ramp", L, check_permutations(code.hz.shape[0], L, 3))
        dec = pk.Decoder(code.hx, code.hz, bx, bz, 20, alpha=0.875, max_batch=shots)
    else:
        wl = WORKLOADS["bb144_L16_T50"]
        code, p, shots, sched = wl.code(), 0.06, 20000, 1
        dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots, schedule=pk.LAYERED)
    dec.set_config(0, 64, 4, 1, 0)  # plain form: one shot per work item
    say(f"plain grid stride {case}: n={code.n} shots={shots}")
    ex, ez, sx, sz = dec.sample(21, p, 0, shots)
    prior = torch.full((code.n,), f32(oracle.prior_llr(p)), dtype=torch.float32, device="cuda")
    a = dec.decode(sx, sz, prior, prior)
    b = dec.decode_batched(sx, sz, prior, prior)
    torch.cuda.synchronize()
    for tag in ("x", "z"):
        np.testing.assert_array_equal(words(a[f"corr_{tag}"]), words(b[f"corr_{tag}"]))
        np.testing.assert_array_equal(a[f"basis_{tag}"].cpu().numpy(), b[f"basis_{tag}"].cpu().numpy())
        np.testing.assert_array_equal(words(a[f"conv_{tag}"]), words(b[f"conv_{tag}"]))
    dec.close()


# ------------------------------------------------------------------ decode statistics

@pytest.mark.parametrize("batched", [0, 1])
def test_decode_stats_equal_run_counters(pk, batched):
    """mbbp_set_stats: a decode call on the sampler's syndromes with the library's
    uniform priors adds the same SUM_K, EDGE_UPDATES, NOCONV and TIES as mbbp_run over
    the same shots, and leaves the other counters alone."""
    wl = WORKLOADS["bb72_L4_T20"]
    code = wl.code()
    shots, p = 5000, 0.05
    dec, bx, bz = make_decoder(pk, code, wl, max_batch=shots)
    ref = dec.run(wl.seed, p, 0, shots)
    ex, ez, sx, sz = dec.sample(wl.seed, p, 0, shots)
    prior = torch.full((code.n,), pk.prior_llr(p), dtype=torch.float32, device="cuda")
    st = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
    dec.set_stats(st)
    (dec.decode_batched if batched else dec.decode)(sx, sz, prior, prior)
    dec.set_stats(None)
    (dec.decode_batched if batched else dec.decode)(sx, sz, prior, prior)  # not counted
    torch.cuda.synchronize()
    got, exp = st.cpu().numpy(), ref.cpu().numpy()
    say(f"decode stats batched={batched}: {got.tolist()} vs run {exp.tolist()}")
    for k in (pk.CNT_SUM_K, pk.CNT_EDGE_UPDATES, pk.CNT_NOCONV, pk.CNT_TIES):
        assert got[k] == exp[k]
    for k in (pk.CNT_FAIL, pk.CNT_FAIL_X, pk.CNT_FAIL_Z, pk.CNT_SUM_KMAX):
        assert got[k] == 0
    dec.close()


# ------------------------------------------------------------------ the known first iteration

@pytest.mark.parametrize("one_per_wave", [False, True])
@pytest.mark.parametrize("T,p,prior_kind", [(0, 0.01, "uniform"), (1, 0.01, "uniform"), (2, 0.03, "uniform"),
                                            (20, 0.005, "uniform"), (20, 0.04, "varying"),
                                            (6, 0.04, "one negative")])
def test_first_iteration_paths_bit_exact(pk, one_per_wave, T, p, prior_kind):
    """Flooding min-sum with one positive prior on every variable starts a shot from
    the first iteration's known outcome (zero syndrome: K = 0 and a zero correction
    without BP; otherwise the first check messages written from the syndrome);
    other prior vectors run that iteration.  Both against the FP32 oracle, bit for
    bit, in the paired and the one-instance kernel, with T = 0, 1, 2 and at error
    rates where many shots have a zero syndrome."""
    wl = WORKLOADS["bb144_L16_T50"]
    code = wl.code()
    shots = 1500
    dec, bx, bz = make_decoder(pk, code, wl, T=T, max_batch=shots, one_per_wave=one_per_wave)
    ex, ez, sx, sz = dec.sample(11, p, 300, shots)
    mu = f32(oracle.prior_llr(p))
    rng = np.random.default_rng(7)
    if prior_kind == "uniform":
        pri = np.full(code.n, mu, dtype=np.float32)
    elif prior_kind == "varying":
        pri = (mu * rng.uniform(0.5, 1.5, code.n)).astype(np.float32)
    else:
        pri = np.full(code.n, mu, dtype=np.float32)
        pri[rng.integers(code.n)] = -mu  # one variable believed flipped: decisions start non-zero
    prior = torch.tensor(pri, dtype=torch.float32, device="cuda")
    say(f"first-iteration paths T={T} p={p} prior={prior_kind} one_per_wave={one_per_wave}")
    for part, h, (bp, rows), syn in ((0, code.hz, bz, sx), (1, code.hx, bx, sz)):
        cand, kstat, _ = dec.decode_detail(part, syn, prior, want_llr=False)
        torch.cuda.synchronize()
        ref = oracle_decode_par(h, bp, rows, words(syn), pri.astype(np.float64), T, alpha=wl.alpha, precision="f32")
        ks = kstat.cpu().numpy().view(np.uint16)
        K, conv = (ks & 0x7FFF).astype(np.int32), (ks >> 15).astype(bool)
        np.testing.assert_array_equal(K, ref.K, err_msg=f"part {part} iterations")
        np.testing.assert_array_equal(conv, ref.conv, err_msg=f"part {part} convergence")
        np.testing.assert_array_equal(words(cand), ref.cand, err_msg=f"part {part} hard decisions")
        zero = int((words(syn) == 0).all(axis=1).sum())
        say(f"  part {part}: zero syndromes {zero} of {shots}, mean K {K.mean():.3f}, converged {conv.mean():.4f}")
    dec.close()
