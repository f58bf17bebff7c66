#!/usr/bin/env python3
"""Throughput of the MBBP-LD hot path on one MI355X.

One step = the whole path over one batch of the [[144,12,12]] workload: for every
error rate p in {0.02, 0.04, 0.06, 0.08}, `shots` (default 10^6) shots of
code-capacity depolarizing noise generated on the GPU, their syndromes, BP
(normalized min-sum, flooding, T = 50, alpha = 0.875) on the 16 subtree
representations of each of H_X and H_Z, the least-weight decision and the
logical-failure test, accumulated into device counters.  Inputs are synthetic
and generated inside the timed region (the noise sampler is one of the path's
steps); nothing is cached between steps (each step decodes fresh shot indices).

Prints one JSON line.  `value` is decoded shots per second; the edge-message
update rate, the roofline of the BP kernel (from HIP events recorded around every
BP launch on its stream) and the CPU oracle baseline ride along.
"""

from __future__ import annotations

import argparse
import concurrent.futures
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU lane-operations per edge-message update of normalized min-sum,
# flooding: v->c exclusion sum 2, sign extract and parity 2, two-minimum tracking 5,
# output select, scaling and sign 4, posterior accumulation 1 (the decision and
# parity bits are bit-packed, under 1).
OPS_PER_EDGE_UPDATE = 14.0
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (non-packed 32-bit VALU lane-ops)
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# LDS: 256 CUs x 128 B/clk x 2.4 GHz; algorithmic LDS bytes per edge update: one
# 4-byte write and one 4-byte read of the exchanged message
LDS_PEAK_TBPS = 256 * 128 * 2.4e9 / 1e12
LDS_BYTES_PER_EDGE_UPDATE = 8.0
# HBM3E
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="bb144_L16_T50")
    ap.add_argument("--shots", type=int, default=None, help="shots per error rate per step")
    ap.add_argument("--form", choices=["batched", "plain", "per-basis"], default="batched",
                    help="batched: mbbp_run (persistent launch, graph replay); plain: sample + mbbp_decode + "
                         "failures; per-basis: the same with one BP launch per (part, representation)")
    ap.add_argument("--rule", choices=["nms", "spa"], default="nms")
    ap.add_argument("--schedule", choices=["flooding", "layered"], default="flooding")
    ap.add_argument("--per-shot-priors", action="store_true",
                    help="non-uniform soft priors per shot and qubit (resident in HBM before the timed region), "
                         "decoded by mbbp_decode_batched")
    ap.add_argument("--lpi", type=int, default=0, help="lanes per BP instance (0 = library choice)")
    ap.add_argument("--wpb", type=int, default=4, help="waves per block (with --lpi)")
    ap.add_argument("--chunk", type=int, default=8, help="shots per work item (with --lpi)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-shots", type=int, default=60000, help="oracle sample: shots per error rate")
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0 = every host core)")
    ap.add_argument("--train-steps", type=int, default=2000, help="weighted workload: Adam steps")
    ap.add_argument("--train-batch", type=int, default=4096, help="weighted workload: shots per Adam step")
    ap.add_argument("--lr", type=float, default=1e-3, help="weighted workload: Adam learning rate")
    ap.add_argument("--val-every", type=int, default=100, help="weighted workload: validate every k steps (0: off)")
    ap.add_argument("--val-shots", type=int, default=200_000, help="weighted workload: validation shots")
    ap.add_argument("--paper-ler", action="store_true",
                    help="logical error rates under the paper's conditions (Section IV): X errors only, "
                         "layered schedule, T = 100, FWS decision, 100 failures per point")
    ap.add_argument("--ler-ps", default="0.03,0.04,0.05,0.06,0.07,0.08", help="--paper-ler: error rates")
    ap.add_argument("--ler-failures", type=int, default=100, help="--paper-ler: failures per point")
    ap.add_argument("--ler-max-shots", type=int, default=50_000_000, help="--paper-ler: shot cap per point")
    ap.add_argument("--ler-bases", choices=["workload", "tree", "random"], default="workload",
                    help="--paper-ler: the workload's bases, or per partition (the maximal subtrees of one "
                         "root order, Algorithm 2) its subtree rows (tree) or as many random rows (random)")
    ap.add_argument("--ler-partitions", type=int, default=1, help="--paper-ler with tree/random: partitions")
    ap.add_argument("--serial-lanes", type=int, default=0, help="serial schedule: shots per wavefront (0 = library)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the BP launch shape of the timed form with mbbp_autotune before the timed region")
    ap.add_argument("--serial-kernel", choices=["auto", "slots", "lanes", "levels"], default="auto",
                    help="serial schedule kernel: eight lanes per shot, one shot per lane, or level-synchronous")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a device-to-device copy of this many bytes (HBM counter calibration)")
    return ap.parse_args()


# sources of the headline BP kernel (the paired kernel's translation unit: its file and
# the headers it includes); the recorded HBM traffic holds only for these as profiled
KERNEL_SOURCES = ("mbbp_bp_dual.hip", "mbbp_bp_rules.h", "mbbp_device.h", "mbbp_wave.h")


def recorded_traffic(workload, shots_per_launch):
    """HBM bytes per BP launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when that summary was taken on another BP kernel source or
    another launch size."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"bp_kernel_{workload}.md")
    csrc = os.path.join(ROOT, "paper_2605_14170_amd", "csrc")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "`")):
            key, _, val = line.partition(":")
            fields[key.strip()] = val.split()[0] if val.split() else ""
    try:
        h = hashlib.sha256()
        for f in KERNEL_SOURCES:
            h.update(open(os.path.join(csrc, f), "rb").read())
        sha = h.hexdigest()
        if fields.get("kernel_source_sha256") != sha or int(fields.get("shots_per_launch", -1)) != shots_per_launch:
            return None
        return float(fields["bp_kernel_hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def build_decoder(pk, wl, code, max_batch, T=None, rule=0, schedule=0):
    from workloads.perms import check_permutations
    perms = lambda h: check_permutations(h.shape[0], max(wl.L, 8), wl.perm_seed)  # noqa: E731
    bx = pk.build_bases(code.hx, wl.basis_mode, wl.L, perms(code.hx))
    bz = pk.build_bases(code.hz, wl.basis_mode, wl.L, perms(code.hz))
    dec = pk.Decoder(code.hx, code.hz, bx, bz, wl.T if T is None else T, alpha=wl.alpha, rule=rule,
                     schedule=schedule, max_batch=max_batch)
    return dec, bx, bz


def cpu_baseline(wl, code, bx, bz, shots_per_p, threads, shot0s, rule=0, schedule=0):
    """The oracle as it stands (FP64, single-threaded per call) on `threads` host
    threads over disjoint shot ranges: at each p the first `shots_per_p` shots the
    GPU decodes in its first timed step (the same shot indices, so the same noise).
    Its failures give the oracle's logical error rate beside the GPU's."""
    import oracle
    chunk = max(1, -(-shots_per_p // threads))
    jobs = []
    for i, p in enumerate(wl.ps):
        for start in range(0, shots_per_p, chunk):
            jobs.append((i, p, shot0s[i] + start, min(chunk, shots_per_p - start)))
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(lambda j: oracle.run(code, bx, bz, wl.seed, j[1], j[2], j[3], wl.T, wl.alpha,
                                               schedule=schedule, rule=rule), jobs))
    dt = time.perf_counter() - t0
    shots = sum(r.shots for r in res)
    edges = sum(r.edge_updates for r in res)
    per_p = {}
    for i, p in enumerate(wl.ps):
        f = sum(r.fails for j, r in zip(jobs, res) if j[0] == i)
        per_p[str(p)] = dict(shots=shots_per_p, fails=f, ler=f / shots_per_p, ler_95=wilson(f, shots_per_p))
    return dict(value=shots / dt, unit="shots/s", cores=threads, kind="oracle",
                edge_updates_per_s=edges / dt, seconds=dt, per_p=per_p,
                sample=f"the first {shots_per_p} shots of the first timed step at each p in {list(wl.ps)} "
                       f"({shots} shots), FP64 oracle, {threads} threads over disjoint shot ranges")


def wilson(k, n, z=1.959963984540054):
    """Wilson 95% interval of a binomial proportion."""
    import math
    if n == 0:
        return (0.0, 1.0)
    ph = k / n
    den = 1 + z * z / n
    c = (ph + z * z / (2 * n)) / den
    h = z * math.sqrt(ph * (1 - ph) / n + z * z / (4 * n * n)) / den
    return (max(0.0, c - h), min(1.0, c + h))


def paper_ler_main(args, wl, code):
    """The paper's experimental conditions (Section IV) on this workload's code and
    bases: X errors only (binary symmetric channel), normalized min-sum with
    alpha = 0.875, layered schedule, at most 100 iterations, FWS decision; at each p,
    batches of shots until the failure count reaches --ler-failures.  One JSON line
    per p (context for the paper's LER curves, not a throughput figure)."""
    import torch
    import paper_2605_14170_amd as pk
    batch = args.shots or 1_000_000
    torch.cuda.set_device(0)
    from workloads.perms import check_permutations
    if args.ler_bases == "workload":
        perms = lambda h: check_permutations(h.shape[0], max(wl.L, 8), wl.perm_seed)  # noqa: E731
        cases = [(None, pk.build_bases(code.hx, wl.basis_mode, wl.L, perms(code.hx)),
                  pk.build_bases(code.hz, wl.basis_mode, wl.L, perms(code.hz)))]
    else:
        # part X (the only one with errors under X-only noise) decodes on the partition
        # of H_Z; part Z takes as many representations of H_X's partition (cycled), as
        # the library runs the same number for both parts
        cases = []
        for k in range(args.ler_partitions):
            bz = partition_bases(pk, code.hz, k, wl.perm_seed, args.ler_bases)
            bx = partition_bases(pk, code.hx, k, wl.perm_seed, args.ler_bases, count=len(bz[0]) - 1)
            cases.append((k, bx, bz))
    rows = []
    for part_k, bx, bz in cases:
        rows += paper_ler_points(args, pk, wl, code, bx, bz, batch, part_k)
    if len(cases) > 1:
        # over the partitions (the paper's Table II): mean and best (lowest) LER per p
        per_p = {}
        for r in rows:
            per_p.setdefault(r["p"], []).append(r)
        summary = {}
        for p_, rs in sorted(per_p.items(), reverse=True):
            lers = [r["ler"] for r in rs]
            summary[str(p_)] = dict(partitions=len(rs), mean_ler=sum(lers) / len(lers), best_ler=min(lers),
                                    worst_ler=max(lers), shots=sum(r["shots"] for r in rs),
                                    failures=sum(r["failures"] for r in rs),
                                    mean_k=sum(r["mean_k"] for r in rs) / len(rs),
                                    mean_L=sum(r["L"] for r in rs) / len(rs))
        print(json.dumps(dict(table="partitions", workload=wl.key, bases=args.ler_bases,
                              partitions=len(cases), per_p=summary)), flush=True)


def partition_bases(pk, h, k, seed, mode, count=None):
    """Bases of partition k: the maximal subtrees of root order pi_k (the library's
    Algorithm 2, pi_0 the identity), one representation [H; H_t] per subtree t
    (tree), or matched random rows (random, the control of the paper's Table II)."""
    from workloads.partitions import matched_random_bases, tree_bases
    from workloads.perms import check_permutations
    m = h.shape[0]
    perm = check_permutations(m, k + 1, seed)[k]
    cs, order, ns = pk.subtrees(h, perm)
    subs = [[int(c) for c in order if cs[c] == t] for t in range(1, ns + 1)]
    if mode == "tree":
        return tree_bases(subs, count)
    return matched_random_bases(subs, m, seed, k, count)


def paper_ler_points(args, pk, wl, code, bx, bz, batch, part_k):
    import torch
    L = len(bx[0]) - 1
    out = []
    dec = pk.Decoder(code.hx, code.hz, bx, bz, 100, schedule=pk.LAYERED, alpha=0.875, select=pk.FWS,
                     max_batch=batch)
    dec.set_noise(pk.X_ONLY)
    if args.serial_lanes:
        dec.set_serial_lanes(args.serial_lanes)
    dec.set_serial_kernel(getattr(pk, "SERIAL_" + args.serial_kernel.upper()))
    for i, p in enumerate(float(x) for x in args.ler_ps.split(",")):
        c = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
        shots = 0
        dec.bp_time(reset=True)
        dec.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while shots < args.ler_max_shots:
            dec.run(wl.seed, p, (i << 40) + shots, batch, c)
            shots += batch
            if int(c[pk.CNT_FAIL]) >= args.ler_failures:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        dec.set_timing(False)
        bp_ms, _ = dec.bp_time(reset=True)
        cc = c.cpu().numpy()
        f = int(cc[pk.CNT_FAIL])
        lo, hi = wilson(f, shots)
        bases = wl.basis_mode if part_k is None else f"{args.ler_bases} partition {part_k}"
        out.append(dict(p=p, ler=f / shots, shots=shots, failures=f, L=L,
                        mean_k=float(cc[pk.CNT_SUM_K]) / (L * shots)))
        print(json.dumps(dict(workload=wl.key, code=wl.key.split("_")[0], noise="x_only", schedule="layered",
                              T=100, alpha=0.875, decision="FWS", L=L, bases=bases, p=p,
                              shots=shots, failures=f, ler=f / shots, ler_95=[lo, hi],
                              mean_kmax=float(cc[pk.CNT_SUM_KMAX]) / shots,
                              # part Z sees no errors (K = 0 there): mean iterations of part X
                              mean_k=float(cc[pk.CNT_SUM_K]) / (L * shots),
                              noconv=int(cc[pk.CNT_NOCONV]), seconds=round(dt, 3), shots_per_s=shots / dt,
                              serial_kernel=args.serial_kernel, serial_lanes=args.serial_lanes,
                              bp_ms=round(bp_ms, 3),
                              edge_updates_per_s_in_bp=float(cc[pk.CNT_EDGE_UPDATES]) / (bp_ms / 1e3))),
              flush=True)
    dec.close()
    return out


def weighted_main(args, wl, code):
    """Weighted decoder: train (alpha, beta) with Adam on fresh shots, then decode
    the same fresh evaluation shots with the learned weights (T = wl.T) and with
    plain normalized min-sum at T = wl.T and T = 50.  One timed step = one
    evaluation pass of the weighted decoder over `shots` shots."""
    import torch
    import paper_2605_14170_amd as pk
    from paper_2605_14170_amd import weighted

    p = wl.ps[0]
    shots = args.shots or wl.shots
    batch, steps = args.train_batch, args.train_steps
    torch.cuda.set_device(0)
    trainer, bx, bz = build_decoder(pk, wl, code, batch)
    print(f"# {wl.key}: training {steps} Adam steps, batch {batch}, lr {args.lr}, p {p}", file=sys.stderr,
          flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()

    def cb(k, v):
        if k % 200 == 0 or k == steps - 1:
            print(f"# step {k} loss {v:.6f}", file=sys.stderr, flush=True)

    # held-out validation shots (a range disjoint from training and evaluation)
    vdec, _, _ = build_decoder(pk, wl, code, args.val_shots, rule=pk.WEIGHTED)
    va = torch.empty((wl.T, wl.L), dtype=torch.float32, device="cuda")
    vb = torch.empty_like(va)
    vdec.set_weights(va, vb)

    def validate(a, b):
        va.copy_(a)
        vb.copy_(b)
        cnt = vdec.run(wl.seed, p, 5 * 10**8, args.val_shots)
        return float(cnt[pk.CNT_FAIL].item()) / args.val_shots

    tr = weighted.train(trainer, seed=wl.seed + 1000, p=p, batch=batch, steps=steps, lr=args.lr,
                        alpha0=wl.alpha, ckpt_every=5, callback=cb,
                        validate=validate if args.val_every > 0 else None, val_every=args.val_every)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    trainer.close()
    vdec.close()
    alpha, beta, losses = tr.alpha, tr.beta, tr.losses
    eval_shot0 = 10**9
    res = {}
    if args.val_every > 0:
        bdec, _, _ = build_decoder(pk, wl, code, shots, rule=pk.WEIGHTED)
        bdec.set_weights(tr.best_alpha.contiguous(), tr.best_beta.contiguous())
        cnt = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
        for k in range(args.steps):
            bdec.run(wl.seed, p, eval_shot0 + k * shots, shots, cnt)
        res[f"weighted_T{wl.T}_best_validation"] = dict(fails=int(cnt[pk.CNT_FAIL].item()), shots=shots * args.steps,
                                                        step=tr.best_step)
        bdec.close()
    wdec, _, _ = build_decoder(pk, wl, code, shots, rule=pk.WEIGHTED)
    wdec.set_weights(alpha.contiguous(), beta.contiguous())
    for k in range(args.warmup):
        wdec.run(wl.seed, p, 10**12 + k * shots, shots)
    torch.cuda.synchronize()
    counters = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
    wdec.bp_time(reset=True)
    wdec.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        wdec.run(wl.seed, p, eval_shot0 + k * shots, shots, counters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    wdec.set_timing(False)
    bp_ms, bp_launches = wdec.bp_time(reset=True)
    c = counters.cpu().numpy()
    total = shots * args.steps
    res[f"weighted_T{wl.T}_final"] = dict(fails=int(c[pk.CNT_FAIL]), shots=total)
    wdec.close()
    for T in (wl.T, 50):
        dec, _, _ = build_decoder(pk, wl, code, shots, T=T)
        cnt = torch.zeros(pk.NUM_COUNTERS, dtype=torch.int64, device="cuda")
        for k in range(args.steps):
            dec.run(wl.seed, p, eval_shot0 + k * shots, shots, cnt)
        torch.cuda.synchronize()
        cc = cnt.cpu().numpy()
        res[f"plain_T{T}"] = dict(fails=int(cc[pk.CNT_FAIL]), shots=total)
        dec.close()
    for v in res.values():
        v["ler"] = v["fails"] / v["shots"]
        v["ci95"] = wilson(v["fails"], v["shots"])
    edges = int(c[pk.CNT_EDGE_UPDATES])
    bp_avg_s = bp_ms / 1e3 / max(1, bp_launches)
    achieved = edges / max(1, bp_launches) * OPS_PER_EDGE_UPDATE / bp_avg_s / 1e12 if bp_launches else None
    line = dict(metric="MBBP-LD decoded shots/s and BP edge-msg updates/s at matched logical error rate",
                value=total / dt, unit="shots/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=dt * 1e3 / args.steps, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", data="synthetic",
                config=dict(workload=wl.key, code=code.name, n=code.n, L=wl.L, T=wl.T, p=p, shots_per_step=shots,
                            rule="weighted min-sum (learned alpha, beta per iteration and representation)",
                            schedule="flooding", eval_shot0=eval_shot0),
                edge_updates_per_s=edges / dt,
                training=dict(steps=steps, batch=batch, lr=args.lr, seconds=train_s,
                              ms_per_adam_step=train_s * 1e3 / max(1, steps), first_loss=losses[0],
                              last_loss=float(np.mean(losses[-20:])), ckpt_every=5,
                              alpha_range=[float(alpha.min()), float(alpha.max())],
                              beta_range=[float(beta.min()), float(beta.max())],
                              validation=[(k, v) for k, v in tr.validation]),
                ler=res,
                roofline=dict(bound="alu", achieved=achieved, peak=VALU_PEAK_TOPS, unit="T lane-op/s",
                              frac=(achieved / VALU_PEAK_TOPS) if achieved else None, traffic=None,
                              kernel="bp_kernel (weighted)", avg_launch_ms=bp_avg_s * 1e3))
    print(json.dumps(line), flush=True)


def algorithmic_hbm_bytes_per_shot(code, form="batched"):
    """Bytes a shot must move to or from HBM.  Errors generated in the kernel: both
    corrections, both convergence masks, both chosen representations and the failure
    flag (about 69 B for n = 144).  Per-shot priors (a decode call): the two prior
    vectors and syndromes in, corrections, masks and representations out (about
    1.25 KB for n = 144)."""
    W = (code.n + 63) // 64
    if form == "pps":
        Ws = (code.hx.shape[0] + 63) // 64
        return 2 * code.n * 4 + 2 * Ws * 8 + 2 * W * 8 + 2 * 8 + 2 * 2
    return 2 * W * 8 + 2 * 8 + 2 * 2 + 1


def soft_priors(torch, code, p, shots, seed):
    """Per-shot, per-qubit priors of a non-uniform channel (inputs of the per-shot
    prior workload): flip probability q of each (shot, qubit, part) drawn
    log-uniformly in [p/3, 4p/3], prior log((1 - q) / q); generated on the GPU before
    the timed region."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    out = []
    for _ in range(2):
        u = torch.rand((shots, code.n), generator=g, device="cuda", dtype=torch.float64)
        q = (p / 3.0) * torch.exp(u * np.log(4.0))
        out.append(torch.log((1.0 - q) / q).to(torch.float32).contiguous())
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); a multi-GPU run "
              f"(shot sharding with one all-reduce of the counters) is not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_bytes:
        # Plain copy kernel of known size: what FETCH_SIZE / WRITE_SIZE read for it
        # calibrates the same counters on the BP kernel.
        x = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_bytes=args.copy_bytes, dispatches=3)))
        return

    import paper_2605_14170_amd as pk
    from workloads.configs import WORKLOADS

    wl = WORKLOADS[args.workload]
    code = wl.code()
    if "weighted" in wl.key:
        return weighted_main(args, wl, code)
    if args.paper_ler:
        return paper_ler_main(args, wl, code)
    shots = args.shots or wl.shots
    rule = pk.SPA if args.rule == "spa" else pk.NMS
    schedule = pk.LAYERED if args.schedule == "layered" else pk.FLOODING
    torch.cuda.set_device(0)
    dec, bx, bz = build_decoder(pk, wl, code, shots, rule=rule, schedule=schedule)
    if args.lpi:
        for form in (0, 1):
            dec.set_config(form, args.lpi, args.wpb, args.chunk, 0)
    form = "pps" if args.per_shot_priors else args.form
    if form == "per-basis":
        dec.set_per_basis(True)
    ps = list(wl.ps)
    if args.autotune:
        tuned = dec.autotune(1 if form in ("batched", "pps") else 0, seed=wl.seed + 77, p=ps[len(ps) // 2],
                             shots=min(shots, 1 << 18))
        print(f"# autotuned launch: {tuned}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    pri = {p: soft_priors(torch, code, p, shots, 1000 + i) for i, p in enumerate(ps)} if form == "pps" else None
    unif = {p: torch.full((code.n,), pk.prior_llr(p), dtype=torch.float32, device="cuda") for p in ps}
    base_of = lambda k, i: (k * len(ps) + i) * shots  # noqa: E731  fresh shot indices per step and p

    def step(k, counters):
        for i, p in enumerate(ps):
            base = base_of(k, i)
            if form == "batched":
                dec.run(wl.seed, p, base, shots, counters[i], stream)
                continue
            ex, ez, sx, sz = dec.sample(wl.seed, p, base, shots, stream)
            px, pz = pri[p] if form == "pps" else (unif[p], unif[p])
            dec.set_stats(counters[i])  # iterations and edge updates of this decode call
            out = (dec.decode_batched if form == "pps" else dec.decode)(sx, sz, px, pz, stream)
            f = dec.failures(ex, ez, out["corr_x"], out["corr_z"], stream)
            counters[i, pk.CNT_FAIL] += (f != 0).sum()

    print(f"# workload {wl.key}: {wl.description}; shots/p/step {shots}; form {form}, rule {args.rule}, "
          f"schedule {args.schedule}", file=sys.stderr, flush=True)
    warm = torch.zeros((len(ps), pk.NUM_COUNTERS), dtype=torch.int64, device="cuda")
    for k in range(args.warmup):
        step(10_000 + k, warm)
    torch.cuda.synchronize()
    print("# warmup done", file=sys.stderr, flush=True)
    counters = torch.zeros((len(ps), pk.NUM_COUNTERS), dtype=torch.int64, device="cuda")
    dec.bp_time(reset=True)
    dec.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, counters)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dec.set_timing(False)
    dec.set_stats(None)
    bp_ms, bp_launches = dec.bp_time(reset=True)
    c = counters.cpu().numpy()
    total_shots = shots * len(ps) * args.steps
    n_per_p = shots * args.steps
    edges = int(c[:, pk.CNT_EDGE_UPDATES].sum())
    ms_per_step = dt * 1e3 / args.steps
    value = total_shots / dt
    per_p = {}
    for i, p in enumerate(ps):
        f = int(c[i, pk.CNT_FAIL])
        d = dict(fails=f, ler=f / n_per_p, ler_95=wilson(f, n_per_p))
        if form == "batched":  # the decode calls report no per-shot maximum
            d.update(mean_kmax=float(c[i, pk.CNT_SUM_KMAX]) / n_per_p)
        d.update(mean_k=float(c[i, pk.CNT_SUM_K]) / (n_per_p * 2 * wl.L),
                 noconv_frac=float(c[i, pk.CNT_NOCONV]) / (n_per_p * 2),
                 ties_frac=float(c[i, pk.CNT_TIES]) / (n_per_p * 2))
        per_p[str(p)] = d
    print(f"# timed {args.steps} steps in {dt:.3f} s; BP kernel {bp_ms:.1f} ms over {bp_launches} launches",
          file=sys.stderr, flush=True)
    if form == "batched" and len(ps) > 1:
        # BP time per error rate, from one more (untimed) call per p after the timed region
        scratch = torch.zeros((1, pk.NUM_COUNTERS), dtype=torch.int64, device="cuda")
        for i, p in enumerate(ps):
            dec.bp_time(reset=True)
            dec.set_timing(True)
            dec.run(wl.seed, p, base_of(0, i), shots, scratch[0], stream)
            torch.cuda.synchronize()
            dec.set_timing(False)
            ms_p, _ = dec.bp_time(reset=True)
            per_p[str(p)]["bp_ms"] = ms_p
        print("# BP ms per error rate: " + ", ".join(f"{p}: {per_p[str(p)]['bp_ms']:.2f}" for p in ps),
              file=sys.stderr, flush=True)
    roofline = None
    launches_per_step = bp_launches / max(1, args.steps)
    bp_avg_s = bp_ms / 1e3 / max(1, bp_launches)
    if edges is not None and bp_launches:
        edges_per_launch = edges / bp_launches
        achieved = edges_per_launch * OPS_PER_EDGE_UPDATE / bp_avg_s / 1e12
        traffic = recorded_traffic(wl.key, shots) if (args.form == "batched" and rule == pk.NMS and
                                                       schedule == pk.FLOODING) else None
        alg_hbm = algorithmic_hbm_bytes_per_shot(code, form) * shots
        lds_tbps = edges_per_launch * LDS_BYTES_PER_EDGE_UPDATE / bp_avg_s / 1e12
        roofline = dict(
            bound="alu", achieved=achieved, peak=VALU_PEAK_TOPS, unit="T lane-op/s", frac=achieved / VALU_PEAK_TOPS,
            traffic=traffic, traffic_unit="HBM bytes per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE, "
                                          "recorded for this kernel source and launch size, else null)",
            kernel="BP kernel", avg_launch_ms=bp_avg_s * 1e3, launches=bp_launches,
            edge_updates_per_launch=edges_per_launch, ops_per_edge_update=OPS_PER_EDGE_UPDATE,
            edge_updates_per_s_in_kernel=edges_per_launch / bp_avg_s,
            lds=dict(algorithmic_bytes_per_edge_update=LDS_BYTES_PER_EDGE_UPDATE, achieved_TBps=lds_tbps,
                     peak_TBps=LDS_PEAK_TBPS, frac=lds_tbps / LDS_PEAK_TBPS),
            hbm=dict(algorithmic_bytes_per_launch=alg_hbm,
                     algorithmic_bytes_per_shot=algorithmic_hbm_bytes_per_shot(code, form),
                     # the algorithmic bytes moved at the BP kernel's rate, and that rate's share of HBM
                     algorithmic_GBps=alg_hbm / bp_avg_s / 1e9,
                     algorithmic_frac=alg_hbm / bp_avg_s / 1e9 / HBM_PEAK_GBPS,
                     achieved_GBps=(traffic / bp_avg_s / 1e9) if traffic else None, peak_GBps=HBM_PEAK_GBPS,
                     frac=(traffic / bp_avg_s / 1e9 / HBM_PEAK_GBPS) if traffic else None,
                     traffic_over_algorithmic=(traffic / alg_hbm) if traffic else None))
    line = dict(metric="MBBP-LD decoded shots/s and BP edge-msg updates/s at matched logical error rate",
                value=value, unit="shots/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
                ms_per_step=ms_per_step, higher_is_better=True, scaling="weak", vs_baseline=None,
                dtype="f32", data="synthetic",
                config=dict(workload=wl.key, code=code.name, n=code.n, L=wl.L, T=wl.T, alpha=wl.alpha,
                            ps=ps, shots_per_p=shots, schedule=args.schedule,
                            rule="sum-product" if rule == pk.SPA else "normalized min-sum",
                            form={"batched": "batched (mbbp_run, persistent launch, graph replay)",
                                  "plain": "plain (mbbp_sample + mbbp_decode + mbbp_failures)",
                                  "per-basis": "plain with one BP launch per (part, representation)",
                                  "pps": "per-shot priors (mbbp_sample + mbbp_decode_batched + mbbp_failures)"}[form],
                            basis_mode=wl.basis_mode, bp_launches_per_step=launches_per_step,
                            launch=dec.get_config(1 if form in ("batched", "pps") else 0)),
                edge_updates_per_s=(edges / dt) if edges is not None else None, per_p=per_p, roofline=roofline)
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or len(os.sched_getaffinity(0))
        print(f"# cpu baseline: oracle on {threads} threads", file=sys.stderr, flush=True)
        import oracle
        from workloads.perms import check_permutations
        obx = oracle.build_bases(code.hx, wl.basis_mode, wl.L,
                                 check_permutations(code.hx.shape[0], max(wl.L, 8), wl.perm_seed))
        obz = oracle.build_bases(code.hz, wl.basis_mode, wl.L,
                                 check_permutations(code.hz.shape[0], max(wl.L, 8), wl.perm_seed))
        n_cpu = min(args.cpu_shots, shots)
        cb = cpu_baseline(wl, code, obx, obz, n_cpu, threads, [base_of(0, i) for i in range(len(ps))],
                          rule=int(rule), schedule=int(schedule))
        line["cpu_baseline"] = cb
        # matched logical error rate: the GPU decodes the oracle's very shots again
        # (outside the timed region) and both failure counts are compared on them
        for i, p in enumerate(ps):
            d, o = per_p[str(p)], cb["per_p"][str(p)]
            g = dec.run(wl.seed, p, base_of(0, i), n_cpu).cpu().numpy()
            gf = int(g[pk.CNT_FAIL])
            d["oracle_sample"] = dict(shots=n_cpu, oracle_fails=o["fails"], oracle_ler=o["ler"],
                                      oracle_ler_95=o["ler_95"], gpu_fails=gf, gpu_ler=gf / n_cpu,
                                      gpu_ler_95=wilson(gf, n_cpu))
            d["gpu_ler_in_oracle_95"] = o["ler_95"][0] <= d["ler"] <= o["ler_95"][1]
    dec.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
