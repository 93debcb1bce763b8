#!/usr/bin/env python3
"""Key-switching benchmark on one MI355X.

Step = one Rotate (Algorithm 3: automorph, Decomp, ModUp, KSKInnerProd,
ModDown x2, add) of an N = 2^16 ciphertext at level L = 24 with K = 8 special
primes and dnum = 3 (one 96 MiB rotation key), through the C ABI.  Inputs are
seeded synthetic uniform residues resident in HBM; the timed loop cycles over
a pool of distinct (ciphertext, key) pairs larger than the 256 MB Infinity
Cache so that every step streams its key from HBM.

Prints ONE JSON line (stdout).  Progress and the per-kernel breakdown go to
stderr.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import contextlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2112_06396_amd import build  # noqa: E402  (source hash of the kernel files; no GPU use)

METRIC = "key-switch ops/s @N=2^16,L=24 (batched vs plain); achieved HBM GB/s; p99 ms"
LOG_N, L, K, DNUM, LEVEL = 16, 24, 8, 3, 24
WORKLOAD = 2  # seed family of this workload

HBM_PEAK_GBS = 8000.0
# Derived peak of the lazy Shoup modular product (the NTT butterfly's
# multiply).  gfx950 compiles it to 5 v_mad_u64_u32 and 12 other 32-bit VALU
# instructions.  Plain 32-bit VALU instructions issue at the fp32 vector
# rate, 157.3 TFLOP/s / 2 / (256 CUs x 4 SIMDs x 2.4 GHz) = 32 lanes per SIMD
# per clock: 2 clocks per 64-wide wave instruction.  v_mad_u64_u32 issues at
# a quarter of that rate (8 clocks; AMD publishes no figure, a probe of
# independent chains measures 20 T/s against 35 T/s for v_fma_f64).  So one wave-wide
# product takes 5 x 8 + 12 x 2 = 64 SIMD clocks: one product per SIMD per
# clock.
SIMDS, CLOCK_HZ = 256 * 4, 2.4e9
MODMUL_CLOCKS_PER_WAVE = 5 * 8 + 12 * 2
MODMUL_PEAK = SIMDS * CLOCK_HZ * 64 / MODMUL_CLOCKS_PER_WAVE


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# launch plans used per workload ("tuned": the package's cache of plans timed
# on this architecture and shape; "default": the library's)
PLANS_USED = {}
USE_TUNED_PLANS = True


@contextlib.contextmanager
def tuned_plan(hks, ctx, workload: str):
    """Inside the block, the context runs the cached tuned plan for
    `workload` (e.g. "batch16_l24") and the context's shape, if the cache has
    one; the previous plan is restored after."""
    import torch
    from paper_2112_06396_amd import tune
    prev = hks.hks_get_plan(ctx)
    entry = None
    if USE_TUNED_PLANS:
        arch = torch.cuda.get_device_properties(0).gcnArchName
        entry = tune.apply_cached(ctx, tune.cache_key(arch, ctx.log_n, ctx.L, ctx.K, ctx.dnum, workload))
    PLANS_USED[workload] = "tuned" if entry else "default"
    try:
        yield
    finally:
        hks.hks_set_plan(ctx, prev)


def kernel_work(cls: int, n: int, level: int, k: int, alpha: int, beta: int):
    """Algorithmic modular multiplications of one Rotate done by kernel class
    `cls` (butterflies for NTT passes, product terms for the conversion and
    KSKInnerProd) and the algorithmic HBM bytes it moves (8-byte words: each
    limb a launch touches read once and written once)."""
    log_n = n.bit_length() - 1
    n1 = log_n // 2
    n2 = log_n - n1
    E = level + k
    new_limbs = beta * E - level  # ModUp's converted limbs (the digits' own limbs are not copied)
    half = n // 2
    if cls == 0:  # forward NTT, column pass: ModUp's new limbs + ModDown's corrections (u and v)
        limbs = new_limbs + 2 * level
        return limbs * half * n1, limbs * n * 16
    if cls == 1:  # forward NTT, row pass of the corrections + ModDown epilogue (reads u, and b for v)
        return 2 * level * half * n2, (2 * level * 16 + 2 * level * 8 + level * 8) * n
    if cls == 2:  # inverse NTT, row pass of the input limbs (automorph gathered)
        return level * half * n2, level * n * 16
    if cls == 3:  # inverse NTT, column pass (+ folded scale on half the outputs): input + P limbs
        limbs = level + 2 * k
        return limbs * half * (n1 + 1), limbs * n * 16
    if cls == 4:  # conversion: ModUp sum_j |I_j| (E - |I_j|) + ModDown 2 K level
        terms = 0
        for j in range(beta):
            sz = min(alpha, level - j * alpha)
            terms += sz * (E - sz)
        terms += 2 * k * level
        return terms * n, (level + new_limbs + 2 * k + 2 * level) * n * 8
    if cls == 5:  # KSKInnerProd fused with ModUp's row pass and ModDown's first inverse pass (P limbs)
        mm = 2 * beta * E * n + new_limbs * half * n2 + 2 * k * half * n2
        words = beta * 2 * E + new_limbs + level + 2 * level + 2 * k  # key, ext, own digits, u/v out, P out
        return mm, words * n * 8
    return 0, 0


def read_traffic(kernel_name: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_name}_rotate_n16_l24_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != build.source_hash():
        return None
    return float(t.group(1))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# CPU baseline workers: each holds one Rotate input of the benchmark workload
# and runs the single-threaded C oracle on it.
_CPU_CASE = None


# the small configuration (N = 2^12, L = 4, K = 2, dnum = 2) and the hoisted
# sample's rotations per call
SMALL = (12, 4, 2, 2)
HROT_SAMPLE = 4


def _cpu_worker_init():
    global _CPU_CASE, _CPU_SMALL
    import numpy as np
    from oracle import oracle as O
    from paper_2112_06396_amd import synth
    pr = O.make_params(LOG_N, L, K, DNUM)
    g = synth.rng(synth.seed_for(WORKLOAD, synth.KIND_CT, 999))
    ct = np.stack([synth.uniform_residues(g, pr.q[:LEVEL], pr.n) for _ in range(2)])
    ksk = np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                    for _ in range(DNUM)])
    _CPU_CASE = (pr, ct, ksk, pow(5, -1, 2 * pr.n))
    O.rotate(pr, ct, LEVEL, _CPU_CASE[3], ksk)  # warm (library loaded, pages touched)
    ps = O.make_params(*SMALL)
    cs = np.stack([synth.uniform_residues(g, ps.q[:SMALL[1]], ps.n) for _ in range(2)])
    ks = np.stack([np.stack([synth.uniform_residues(g, ps.key_mods(), ps.n) for _ in range(2)])
                   for _ in range(SMALL[3])])
    _CPU_SMALL = (ps, cs, ks, pow(5, -1, 2 * ps.n))


def _cpu_worker_rotates(count: int) -> int:
    from oracle import oracle as O
    pr, ct, ksk, gal = _CPU_CASE
    for _ in range(count):
        O.rotate(pr, ct, LEVEL, gal, ksk)
    return count


def _cpu_worker_job(job) -> int:
    """(kind, count): count calls of the small Rotate ("c1") or of an
    HRotate over HROT_SAMPLE rotations at the benchmark's shape ("c3a", one
    key for every rotation: the oracle's cost does not depend on key values);
    returns the key-switches done."""
    from oracle import oracle as O
    kind, count = job
    if kind == "c1":
        ps, cs, ks, gal = _CPU_SMALL
        for _ in range(count):
            O.rotate(ps, cs, SMALL[1], gal, ks)
        return count
    pr, ct, ksk, _ = _CPU_CASE
    gals = [pow(5, k + 1, 2 * pr.n) for k in range(HROT_SAMPLE)]
    for _ in range(count):
        O.hrotate(pr, ct, LEVEL, gals, [ksk] * HROT_SAMPLE)
    return count * HROT_SAMPLE


def cpu_baseline(per_worker: int, workers: int):
    """The plain C oracle (single-threaded, unchanged) on the benchmark's
    Rotate: one host core, and `workers` cores each running the oracle in a
    process of its own; three timed runs each, median reported.  Started
    before the GPU is touched (workers are spawned from a clean process)."""
    import multiprocessing as mp
    import statistics
    ctx = mp.get_context("spawn")
    res = {}
    with ctx.Pool(workers, initializer=_cpu_worker_init) as pool:
        pool.map(_cpu_worker_rotates, [0] * workers)  # every worker initialized
        one, many = [], []
        for _ in range(3):
            t0 = time.perf_counter()
            pool.apply(_cpu_worker_rotates, (per_worker,))
            one.append(per_worker / (time.perf_counter() - t0))
        for _ in range(3):
            t0 = time.perf_counter()
            done = sum(pool.map(_cpu_worker_rotates, [per_worker] * workers, chunksize=1))
            many.append(done / (time.perf_counter() - t0))
        def timed(kind, count):
            """Median over 3 runs of the key-switches/s on one core and on all
            `workers` cores."""
            o, m = [], []
            for _ in range(3):
                t0 = time.perf_counter()
                done = pool.apply(_cpu_worker_job, ((kind, count),))
                o.append(done / (time.perf_counter() - t0))
            for _ in range(3):
                t0 = time.perf_counter()
                done = sum(pool.map(_cpu_worker_job, [(kind, count)] * workers, chunksize=1))
                m.append(done / (time.perf_counter() - t0))
            return {"value": statistics.median(m), "runs": m, "single_core": statistics.median(o),
                    "single_core_runs": o}
        small = timed("c1", 40)
        hoisted = timed("c3a", 1)
    res = {"value": statistics.median(many), "unit": "key-switch/s", "cores": workers, "kind": "oracle",
           "sample": f"3 timed runs of {workers} x {per_worker} Rotate calls at N=2^16, L=24, K=8, dnum=3, one "
                     f"single-threaded C-oracle process per core; median of the runs' throughputs",
           "runs": many, "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "single_core": {"value": statistics.median(one), "runs": one,
                           "sample": f"3 timed runs of {per_worker} Rotate calls on one core"},
           "other_configs": {
               "C1_small_rotate": dict(small, unit="key-switch/s",
                                       sample="3 timed runs of 40 Rotate calls at N=2^12, L=4, K=2, dnum=2 per "
                                              "core (all cores, and one core)"),
               "C3a_hoisted": dict(hoisted, unit="rotations/s",
                                   sample=f"3 timed runs of one HRotate over {HROT_SAMPLE} rotations at N=2^16, "
                                          f"L=24, K=8, dnum=3 per core (ModUp once per call; the 64-rotation "
                                          f"form amortizes it further)"),
               "C3b_batch": {"note": "32 independent Rotates: the oracle's rate is the plain Rotate's above"},
               "C4_trace": {"note": "not timed: the 120 key-switches at L = 35 -> 9 take minutes on the oracle; "
                                    "each costs about a plain Rotate at its level"}}}
    return res


def extras(args, ctx, hks, synth, cts, ksks, outs, gal, key_mods, n, plain_value, stream):
    """Batched, hoisted, graph-replayed and trace figures beside the plain
    Rotate: the same N=2^16, L=24, dnum=3 key-switch in the forms of the
    paper's hoisting / batching and of a bootstrapping-shaped trace."""
    import torch
    from paper_2112_06396_amd import trace
    res = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def rate(fn, per_call, reps):
        fn(0)
        torch.cuda.synchronize()
        e0.record(stream)
        for i in range(reps):
            fn(i + 1)
        e1.record(stream)
        torch.cuda.synchronize()
        return reps * per_call / (e0.elapsed_time(e1) / 1e3)

    # keys and ciphertexts drawn on the GPU (values only need to be residues)
    nk = 64
    dkeys = [synth.device_residues(key_mods, (DNUM, 2), n, 5000 + i) for i in range(nk)]
    dcts = [synth.device_residues(key_mods[:LEVEL], (2,), n, 7000 + i) for i in range(32)]
    douts = [hks.empty((2, LEVEL, n)) for _ in range(nk)]
    gals = [hks.hks_galois_for_rotation(k + 1, LOG_N) for k in range(nk)]
    torch.cuda.synchronize()
    log(f"[bench] extras: {nk} keys, 32 ciphertexts resident")

    # hoisted rotations (Algorithm 4): one ModUp shared by 64 rotations with distinct keys
    with tuned_plan(hks, ctx, f"hrotate{nk}_l{LEVEL}"):
        res["hrotate_r64_ks_per_s"] = rate(
            lambda i: hks.hks_hrotate(ctx, cts[i % args.pool], LEVEL, gals, dkeys, douts, stream), nk, 4)
    # 32 ciphertexts rotated once: one shared key (read once per step) / 32 distinct keys and indices
    with tuned_plan(hks, ctx, f"batch{args.batch}_l{LEVEL}"):
        res["batch32_shared_key_ks_per_s"] = rate(
            lambda i: hks.hks_batch_rotate(ctx, dcts, LEVEL, [gal] * 32, [dkeys[i % nk]] * 32, douts[:32],
                                           stream), 32, 8)
        res["batch32_distinct_keys_ks_per_s"] = rate(
            lambda i: hks.hks_batch_rotate(ctx, dcts, LEVEL, gals[:32], dkeys[32 * (i % 2):32 * (i % 2) + 32],
                                           douts[:32], stream), 32, 8)
    if plain_value:
        res["batch_vs_plain"] = res["batch32_shared_key_ks_per_s"] / plain_value

    # the key-switch kernel's achieved HBM rate in the batched and hoisted
    # forms (separate pass with the library's per-launch events):
    # algorithmic bytes of the launches / their summed durations
    kcls = hks.HKS_K_NAMES.index("ksk")
    alpha, beta = ctx.alpha, ctx.beta(LEVEL)

    def ksk_rate(fn, reps, bytes_of):
        fn(0)
        torch.cuda.synchronize()
        hks.hks_prof_enable(ctx, 1 << kcls)
        for i in range(reps):
            fn(i + 1)
        torch.cuda.synchronize()
        ms, cnt = hks.hks_prof_read(ctx, kcls)
        hks.hks_prof_enable(ctx, 0)
        gbs = bytes_of(reps, cnt) / (ms / 1e3) / 1e9
        return {"achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                "avg_launch_us": ms * 1e3 / cnt, "launches": cnt / reps}

    E = LEVEL + K
    per_rot = kernel_work(kcls, n, LEVEL, K, alpha, beta)[1]  # key, digits, own limbs, u/v, P limbs
    # HRotate: the beta digits of E limbs (converted + own) are shared by the
    # rotations of a launch and count once per launch
    shared = beta * E * n * 8
    forms = {}
    with tuned_plan(hks, ctx, f"batch{args.batch}_l{LEVEL}"):
        forms["batch32_distinct_keys"] = ksk_rate(
            lambda i: hks.hks_batch_rotate(ctx, dcts, LEVEL, gals[:32], dkeys[32 * (i % 2):32 * (i % 2) + 32],
                                           douts[:32], stream), 4, lambda reps, cnt: reps * 32 * per_rot)
    with tuned_plan(hks, ctx, f"hrotate{nk}_l{LEVEL}"):
        forms["hrotate_r64"] = ksk_rate(
            lambda i: hks.hks_hrotate(ctx, cts[i % args.pool], LEVEL, gals, dkeys, douts, stream), 4,
            lambda reps, cnt: reps * nk * (per_rot - shared) + cnt * shared)
    forms["batch32_distinct_keys"]["algorithmic_bytes_per_rotation"] = per_rot
    forms["hrotate_r64"]["algorithmic_bytes_per_rotation"] = per_rot - shared
    forms["hrotate_r64"]["shared_bytes_per_launch"] = shared
    res["ksk_roofline_batched"] = forms
    log(f"[bench] ksk kernel HBM rate: batch 32 distinct keys "
        f"{forms['batch32_distinct_keys']['achieved']:.0f} GB/s, hrotate r=64 {forms['hrotate_r64']['achieved']:.0f} GB/s")
    # the key-streaming step alone (KSKInnerProd, hks_ksk_inner: digits already
    # in evaluation form, 16 keys cycled): key, digits and u, v once each
    exts = [synth.device_residues(key_mods[:LEVEL] + key_mods[L:], (beta,), n, 8000 + i) for i in range(4)]
    uv_d = hks.empty((2, E, n))
    ks_rate = rate(lambda i: hks.hks_ksk_inner(ctx, exts[i % 4], LEVEL, dkeys[i % 16], uv_d, stream), 1, 64)
    ks_bytes = (beta * 2 * E + beta * E + 2 * E) * n * 8
    res["ksk_inner_alone"] = {"us_per_call": 1e6 / ks_rate, "bytes_per_call": ks_bytes,
                              "achieved": ks_rate * ks_bytes / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": ks_rate * ks_bytes / 1e9 / HBM_PEAK_GBS}
    del exts, uv_d
    log(f"[bench] KSKInnerProd alone: {res['ksk_inner_alone']['achieved']:.0f} GB/s "
        f"({100 * res['ksk_inner_alone']['frac']:.0f}% of 8 TB/s)")
    if args.batched_only:
        return res
    # seeded keys (rows a_j regenerated on chip, half the key bytes)
    b_rows = [k[:, 1].contiguous() for k in dkeys[:32]]
    res["rotate_seeded_ks_per_s"] = rate(
        lambda i: hks.hks_rotate_seeded(ctx, cts[i % args.pool], LEVEL, gal, 77 + i % 32, b_rows[i % 32],
                                        outs[i % args.pool], stream), 1, max(50, args.steps))
    res["batch32_seeded_keys_ks_per_s"] = rate(
        lambda i: hks.hks_batch_rotate_seeded(ctx, dcts, LEVEL, gals[:32], [77 + j for j in range(32)], b_rows,
                                              douts[:32], stream), 32, 8)
    del b_rows
    # PtMatVecMult over 12 rotations: the ModDown hoisted (one fused launch, one ModDown) vs
    # HRotate + PtMult + Add (a ModDown per rotation)
    r = 12
    pts = [synth.device_residues(key_mods[:LEVEL] + key_mods[L:], (), n, 9000 + i) for i in range(r)]
    pts_q = [p_[:LEVEL].contiguous() for p_ in pts]
    mv_out = hks.empty((2, LEVEL, n))
    tmp = [hks.empty((2, LEVEL, n)) for _ in range(2)]

    def unhoisted(i):
        hks.hks_hrotate(ctx, cts[i % args.pool], LEVEL, gals[:r], dkeys[:r], douts[:r], stream)
        hks.hks_ptmult(ctx, douts[0], pts_q[0], LEVEL, False, tmp[0], stream)
        for j in range(1, r):
            hks.hks_ptmult(ctx, douts[j], pts_q[j], LEVEL, False, tmp[1], stream)
            hks.hks_add(ctx, tmp[0], tmp[1], LEVEL, 2, tmp[0], stream)

    res["ptmatvec_r12_rot_per_s"] = rate(
        lambda i: hks.hks_ptmatvec(ctx, cts[i % args.pool], LEVEL, gals[:r], dkeys[:r], pts, mv_out, stream), r, 8)
    res["ptmatvec_r12_unhoisted_rot_per_s"] = rate(unhoisted, r, 8)
    del pts, pts_q, mv_out, tmp
    # Mult + relinearization + Rescale vs NewMult (the key-switch ModDown and Rescale merged)
    mrlk = dkeys[0]
    mout = [hks.empty((2, LEVEL - 1, n)) for _ in range(2)]
    res["mult_rescale_per_s"] = rate(
        lambda i: hks.hks_mult_relin(ctx, dcts[i % 32], dcts[(i + 1) % 32], LEVEL, mrlk, True, mout[i % 2], stream),
        1, max(50, args.steps))
    res["new_mult_per_s"] = rate(
        lambda i: hks.hks_new_mult(ctx, dcts[i % 32], dcts[(i + 1) % 32], LEVEL, mrlk, mout[i % 2], stream),
        1, max(50, args.steps))
    log(f"[bench] Mult+Rescale {res['mult_rescale_per_s']:.0f}/s, NewMult {res['new_mult_per_s']:.0f}/s")
    del mout
    # the plain Rotate replayed from hipGraphs (one per pool entry)
    graphs = []
    for j in range(args.pool):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            hks.hks_rotate(ctx, cts[j], LEVEL, gal, ksks[j], outs[j])
        graphs.append(g)
    torch.cuda.synchronize()
    res["graph_rotate_ks_per_s"] = rate(lambda i: graphs[i % args.pool].replay(), 1, max(50, args.steps))
    del graphs
    # the small configuration (N = 2^12, L = 4, K = 2, dnum = 2): latency-bound,
    # a pool of 64 ciphertexts rotated one at a time, eager and from a hipGraph
    sq = hks.hks_gen_primes(50, 13, 6)
    sctx = hks.Context(12, sq[:4], sq[4:], 2)
    scts = [synth.device_residues(sq[:4], (2,), 1 << 12, 60000 + i) for i in range(64)]
    skey = synth.device_residues(sq, (2, 2), 1 << 12, 60100)
    souts = [hks.empty((2, 4, 1 << 12)) for _ in range(64)]
    sgal = hks.hks_galois_for_rotation(1, 12)
    us_eager = 1e6 / rate(lambda i: hks.hks_rotate(sctx, scts[i % 64], 4, sgal, skey, souts[i % 64], stream), 1, 500)
    sg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(sg):
        for j in range(64):
            hks.hks_rotate(sctx, scts[j], 4, sgal, skey, souts[j])
    torch.cuda.synchronize()
    us_graph = 1e6 / rate(lambda i: sg.replay(), 64, 8)
    res["small_rotate"] = {"config": {"log_n": 12, "L": 4, "K": 2, "dnum": 2}, "launches_per_rotate": 9,
                           "us_per_rotate_eager": us_eager, "us_per_rotate_graph": us_graph}
    del sg, scts, souts, skey
    torch.cuda.synchronize()
    sctx.close()
    log(f"[bench] N=2^12 L=4 Rotate: {us_eager:.1f} us eager, {us_graph:.1f} us from a graph of 64")
    log(f"[bench] hrotate r=64 {res['hrotate_r64_ks_per_s']:.0f} ks/s; batch 32 shared key "
        f"{res['batch32_shared_key_ks_per_s']:.0f}, distinct keys {res['batch32_distinct_keys_ks_per_s']:.0f}, "
        f"distinct seeded keys {res['batch32_seeded_keys_ks_per_s']:.0f}; seeded Rotate "
        f"{res['rotate_seeded_ks_per_s']:.0f}; PtMatVecMult r=12 {res['ptmatvec_r12_rot_per_s']:.0f} rot/s "
        f"(unhoisted {res['ptmatvec_r12_unhoisted_rot_per_s']:.0f}); "
        f"graph-replayed Rotate {res['graph_rotate_ks_per_s']:.0f}")
    del dkeys, dcts, douts
    torch.cuda.empty_cache()

    # bootstrapping-shaped trace: L = 35 -> 9, K = 12, dnum = 3, 120 key-switches
    pq = hks.hks_gen_primes(50, LOG_N + 1, 47)
    tctx = hks.Context(LOG_N, pq[:35], pq[35:], 3, max_batch=16)
    plan = trace.bootstrap_plan(35)
    bufs = trace.TraceBuffers(plan, n)
    bufs.view("x0", 35).copy_(synth.device_residues(pq[:35], (2,), n, 11))
    diag = {d: synth.device_residues(pq[:35], (), n, 100 + i) for i, d in enumerate(plan.diagonals)}
    tkeys = {k: synth.device_residues(pq, (3, 2), n, 2000 + i) for i, k in enumerate(plan.rotations)}
    rlk = synth.device_residues(pq, (3, 2), n, 1999)
    with tuned_plan(hks, tctx, "trace_l35"):
        res["trace_ks_per_s_eager"] = rate(lambda i: trace.run_plan(tctx, plan, bufs, diag, tkeys, rlk),
                                           plan.key_switches, 3)
        gr = trace.capture(tctx, plan, bufs, diag, tkeys, rlk)
    res["trace_ks_per_s_graph"] = rate(lambda i: gr.replay(), plan.key_switches, 3)
    res["trace"] = {"key_switches": plan.key_switches, "rotation_keys": len(plan.rotations), "levels": "35->9",
                    "ops": len(plan.ops)}
    del gr
    # the same trace with each linear stage as one PtMatVecMult (ModDown hoisted) and the
    # EvalMod products as NewMult (one ModDown by P q_(l-1))
    hplan = trace.bootstrap_plan(35, hoisted=True, new_mult=True)
    hdiag = {d: synth.device_residues(pq, (), n, 100 + i) for i, d in enumerate(hplan.diagonals)}
    hext = trace.ext_diagonals(hplan, hdiag, 35)
    hbufs = trace.TraceBuffers(hplan, n)
    hbufs.view("x0", 35).copy_(bufs.view("x0", 35))
    with tuned_plan(hks, tctx, "hoisted_trace_l35"):
        res["trace_hoisted_ks_per_s_eager"] = rate(
            lambda i: trace.run_plan(tctx, hplan, hbufs, hdiag, tkeys, rlk, diag_ext=hext), hplan.key_switches, 3)
        gr = trace.capture(tctx, hplan, hbufs, hdiag, tkeys, rlk, diag_ext=hext)
    res["trace_hoisted_ks_per_s_graph"] = rate(lambda i: gr.replay(), hplan.key_switches, 3)
    log(f"[bench] hoisted trace: eager {res['trace_hoisted_ks_per_s_eager']:.0f} ks/s, "
        f"graph {res['trace_hoisted_ks_per_s_graph']:.0f} ks/s")
    del hdiag, hext, hbufs
    log(f"[bench] trace ({plan.key_switches} key-switches, L 35->9): eager {res['trace_ks_per_s_eager']:.0f} ks/s, "
        f"graph {res['trace_ks_per_s_graph']:.0f} ks/s")
    del gr, bufs, diag, tkeys
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # the trace with the factored DFT's own rotation offsets (2^15 slots, fftIter = 3: CoeffToSlot
    # 32/63/63 diagonals, SlotToCoeff 63/63/32, 155 rotation keys resident), diagonals encoded on the
    # device from random slot vectors; hoisted PtMatVecMult + NewMult vs HRotate + PtMult + Mult
    dplan = trace.bootstrap_plan(35, hoisted=True, new_mult=True, dft=(LOG_N - 1, 3))
    dkeys = {k: synth.device_residues(pq, (3, 2), n, 4000 + i) for i, k in enumerate(dplan.rotations)}
    gz = torch.Generator(device="cuda")
    gz.manual_seed(12)
    ddiag = {}
    for d in dplan.diagonals:
        zs = torch.rand((n // 2, 2), generator=gz, dtype=torch.float64, device="cuda") * 2 - 1
        ddiag[d] = hks.empty((len(pq), n))
        hks.hks_encode(tctx, zs, 2.0 ** 40, 35, True, ddiag[d])
    dext = trace.ext_diagonals(dplan, ddiag, 35)
    dbufs = trace.TraceBuffers(dplan, n)
    dbufs.view("x0", 35).copy_(synth.device_residues(pq[:35], (2,), n, 13))
    torch.cuda.synchronize()
    log(f"[bench] DFT trace: {len(dkeys)} rotation keys, {len(ddiag)} encoded diagonals resident")
    with tuned_plan(hks, tctx, "dft_trace_l35"):
        res["dft_trace_ks_per_s_eager"] = rate(
            lambda i: trace.run_plan(tctx, dplan, dbufs, {}, dkeys, rlk, diag_ext=dext), dplan.key_switches, 3)
        gr = trace.capture(tctx, dplan, dbufs, {}, dkeys, rlk, diag_ext=dext)
    res["dft_trace_ks_per_s_graph"] = rate(lambda i: gr.replay(), dplan.key_switches, 3)
    del gr, dext, dbufs
    uplan = trace.bootstrap_plan(35, dft=(LOG_N - 1, 3))
    ubufs = trace.TraceBuffers(uplan, n)
    ubufs.view("x0", 35).copy_(synth.device_residues(pq[:35], (2,), n, 13))
    res["dft_trace_unhoisted_ks_per_s_eager"] = rate(
        lambda i: trace.run_plan(tctx, uplan, ubufs, ddiag, dkeys, rlk), uplan.key_switches, 2)
    res["dft_trace"] = {"key_switches": dplan.key_switches, "rotation_keys": len(dplan.rotations),
                        "diagonals": [len(op[3]) for op in dplan.ops if op[0] == "ptmatvec"], "levels": "35->9"}
    log(f"[bench] DFT trace ({dplan.key_switches} key-switches): hoisted + NewMult eager "
        f"{res['dft_trace_ks_per_s_eager']:.0f} ks/s, graph {res['dft_trace_ks_per_s_graph']:.0f}; "
        f"HRotate + PtMult + Mult {res['dft_trace_unhoisted_ks_per_s_eager']:.0f}")
    del ubufs, ddiag, dkeys, rlk
    torch.cuda.synchronize()
    tctx.close()
    torch.cuda.empty_cache()
    res["w32"] = w32_extra(args, hks, synth, torch.cuda.current_stream())
    res["serving"] = serving_extra(args, hks, synth)
    return res


def w32_extra(args, hks, synth, stream):
    """The same Rotate in 32-bit words (Sec. 5.4): N = 2^16, 30-bit primes,
    L = 40, K = 14, dnum = 3 (log2 QP = 1620 bits against 1600 for the 50-bit
    L = 24, K = 8), level 40, a pool of (ciphertext, key) pairs as for the
    main line; and HRotate over 64 distinct keys as for the 64-bit extra."""
    import torch
    L32, K32 = 40, 14
    pq = hks.hks_gen_primes(30, LOG_N + 1, L32 + K32)
    c32 = hks.Context32(LOG_N, pq[:L32], pq[L32:], DNUM)
    n = 1 << LOG_N

    def d32(mods, lead, seed):
        return synth.device_residues(mods, lead, n, seed).view(torch.int64).to(torch.int32)

    cts = [d32(pq[:L32], (2,), 9100 + i) for i in range(args.pool)]
    keys = [d32(pq, (DNUM, 2), 9200 + i) for i in range(args.pool)]
    outs = [hks.empty32((2, L32, n)) for _ in range(args.pool)]
    gal = hks.hks_galois_for_rotation(1, LOG_N)

    def step(i):
        j = i % args.pool
        hks.hks32_rotate(c32, cts[j], L32, gal, keys[j], outs[j], stream)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        step(i)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    key_bytes = keys[0].numel() * 4
    compulsory = key_bytes + 2 * cts[0].numel() * 4
    del keys, outs
    # hoisted rotations (Algorithm 4): one ModUp shared by 64 rotations with distinct keys
    nk, reps = 64, 4
    hkeys = [d32(pq, (DNUM, 2), 9300 + i) for i in range(nk)]
    houts = [hks.empty32((2, L32, n)) for _ in range(nk)]
    hgals = [hks.hks_galois_for_rotation(k + 1, LOG_N) for k in range(nk)]
    hks.hks32_hrotate(c32, cts[0], L32, hgals, hkeys, houts, stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for i in range(reps):
        hks.hks32_hrotate(c32, cts[(i + 1) % args.pool], L32, hgals, hkeys, houts, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    hrot = reps * nk / (e0.elapsed_time(e1) / 1e3)
    del cts, hkeys, houts
    torch.cuda.synchronize()
    c32.close()
    torch.cuda.empty_cache()
    log(f"[bench] 32-bit words (L=40, K=14, 30-bit primes): {ms * 1e3:.1f} us/step, {1e3 / ms:.0f} ks/s; "
        f"hrotate r=64 {hrot:.0f} ks/s")
    return {"rotate_ks_per_s": 1e3 / ms, "us_per_step": ms * 1e3, "hrotate_r64_ks_per_s": hrot,
            "key_mib": key_bytes / 2 ** 20, "hbm_compulsory_bytes_per_step": compulsory,
            "config": {"log_n": LOG_N, "L": L32, "K": K32, "dnum": DNUM, "level": L32, "prime_bits": 30}}


def serving_extra(args, hks, synth):
    """Continuous batching vs one request at a time for Poisson arrivals of
    Rotate / Mult+relin requests from per-client keys at N in {2^15, 2^16},
    level uniform in [3, 35], L_max = 35, K = 12, dnum = 3.  The keys are
    seeded (Sec. 5.3): only their rows b_j are stored, uploaded and read, the
    rows a_j regenerated on chip (--serving-full-keys: full keys).  Two key
    budgets: every key resident in HBM once touched (the 32 GiB budget of
    the workload, above the seeded key set: the GPU-bound figure), and a
    budget below the key set (LRU eviction, re-upload from pinned host
    memory over PCIe)."""
    import torch
    from paper_2112_06396_amd import serving
    n_clients = args.serving_clients
    seeds = None if args.serving_full_keys else {}
    params = {}
    for ln in (15, 16):
        pq = hks.hks_gen_primes(50, ln + 1, 47)
        params[ln] = (pq[:35], pq[35:], 3)
    host_keys = {}
    for c in range(n_clients):
        ln = 15 if c % 2 == 0 else 16
        q, p, _ = params[ln]
        for j, kind in enumerate(("rot", "rlk")):
            lead = (3,) if seeds is not None else (3, 2)
            d = synth.device_residues(q + p, lead, 1 << ln, 30000 + 2 * c + j)
            if seeds is not None:
                seeds[(c, kind, ln)] = 0x5EED0000 + 2 * c + j
            h = torch.empty(d.shape, dtype=torch.int64, pin_memory=True).view(torch.uint64)
            h.copy_(d)
            host_keys[(c, kind, ln)] = h
            del d
    inputs = {(ln, lv): [synth.device_residues(params[ln][0][:lv], (2,), 1 << ln, 40000 + 100 * lv + 10 * ln + i)
                         for i in range(2)] for ln in (15, 16) for lv in range(3, 36)}
    torch.cuda.synchronize()
    key_bytes = sum(t.numel() * 8 for t in host_keys.values())
    out = {"clients": n_clients, "key_format": "seeded (rows b_j)" if seeds else "full",
           "key_gib": round(key_bytes / 2**30, 1), "grouping": "(N, op), any levels per step", "configs": []}
    for name, budget_gib, n_req in (("resident", args.serving_resident_gib, args.serving_requests),
                                    ("evicting", args.serving_budget_gib, args.serving_requests_evict)):
        if n_req <= 0:
            continue
        ks = serving.KeyStore(host_keys, budget=budget_gib << 30)
        ex = serving.HksExecutor(params, lanes=args.serving_lanes, max_batch=args.batch, slots_per_n=64,
                                 keystore=ks, inputs=inputs, seeds=seeds)
        eng = serving.Engine(ex, lanes=args.serving_lanes, max_batch=args.batch)
        log(f"[bench] serving ({name}): {n_clients} clients, {key_bytes / 2**30:.1f} GiB of "
            f"{'seeded ' if seeds else ''}keys, budget {budget_gib} GiB, {n_req} requests per run")
        if key_bytes <= (budget_gib << 30):
            ks.preload(torch.cuda.current_stream())  # every key resident before the first run
        # capacity of the plain loop: everything arrives at once, one request at a time
        sat = serving.poisson_requests(min(n_req, 2000), rate=1e9, n_clients=n_clients, seed=1)
        cap = eng.run(sat, one_at_a_time=True)["throughput_per_s"]
        sat_b = serving.poisson_requests(min(n_req, 2000), rate=1e9, n_clients=n_clients, seed=1)
        cap_b = eng.run(sat_b)["throughput_per_s"]
        cfg = {"name": name, "key_budget_gib": budget_gib, "all_keys_fit": key_bytes <= (budget_gib << 30),
               "requests_per_run": n_req, "plain_capacity_per_s": cap, "batched_capacity_per_s": cap_b,
               "runs": []}
        log(f"[bench] serving ({name}): capacity {cap:.0f}/s one at a time, {cap_b:.0f}/s batched")
        for f in (0.5, 0.8, 1.0, 1.2):
            row = {"load": f}
            for mode in ("plain", "batched"):
                reqs = serving.poisson_requests(n_req, rate=f * cap, n_clients=n_clients, seed=int(100 * f))
                up0 = ks.uploads
                st = eng.run(reqs, one_at_a_time=(mode == "plain"))
                st["key_uploads"] = ks.uploads - up0
                row[mode] = st
            row["batched_vs_plain_throughput"] = row["batched"]["throughput_per_s"] / row["plain"]["throughput_per_s"]
            cfg["runs"].append(row)
            log(f"[bench] serving ({name}) load {f}: plain {row['plain']['throughput_per_s']:.0f}/s p50 "
                f"{row['plain']['p50_ms']:.2f} p99 {row['plain']['p99_ms']:.2f} ms | batched "
                f"{row['batched']['throughput_per_s']:.0f}/s p50 {row['batched']['p50_ms']:.2f} p99 "
                f"{row['batched']['p99_ms']:.2f} ms")
        ex.close()
        del ks, ex, eng
        torch.cuda.empty_cache()
        out["configs"].append(cfg)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--pool", type=int, default=8)
    ap.add_argument("--batch", type=int, default=16, help="ciphertexts per batched launch step (extras)")
    ap.add_argument("--serving-clients", type=int, default=256)
    ap.add_argument("--serving-budget-gib", type=int, default=16,
                    help="key budget of the evicting serving runs (below the key set)")
    ap.add_argument("--serving-resident-gib", type=int, default=32,
                    help="key budget of the resident serving runs (the workload's 32 GiB)")
    ap.add_argument("--serving-requests", type=int, default=20000, help="requests per resident serving run")
    ap.add_argument("--serving-requests-evict", type=int, default=4000,
                    help="requests per evicting serving run (PCIe-bound; 0 skips them)")
    ap.add_argument("--serving-lanes", type=int, default=2)
    ap.add_argument("--serving-full-keys", action="store_true",
                    help="serve with full keys instead of seeded ones (rows a_j and b_j stored and uploaded; "
                         "256 clients then need 53 GiB of pinned host memory)")
    ap.add_argument("--cpu-sample", type=int, default=2, help="oracle Rotates per core per timed run")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host cores for the all-cores oracle figure (the GPU box grants 16)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving figures (with the --serving-* sizes) and print them")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the hoisted and batched Rotate figures (for profiling) and print them")
    ap.add_argument("--w32-only", action="store_true",
                    help="time only the 32-bit-word Rotate (for profiling) and print its figures")
    ap.add_argument("--default-plans", action="store_true",
                    help="run every figure with the library's default launch plan (no tuned plans)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one plain copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    global USE_TUNED_PLANS
    USE_TUNED_PLANS = not args.default_plans

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the key-switching path runs on a single MI355X "
              "(how it would shard over several GPUs is described, not implemented). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    cpu = None
    if not (args.no_cpu_baseline or args.w32_only or args.serving_only or args.batched_only):
        # before any GPU use: the oracle's worker processes start from a clean process
        log(f"[bench] timing the CPU oracle: {args.cpu_workers} cores x {args.cpu_sample} Rotates, 3 runs")
        cpu = cpu_baseline(args.cpu_sample, args.cpu_workers)
        log(f"[bench] CPU oracle: {cpu['value']:.2f} Rotates/s on {cpu['cores']} cores, "
            f"{cpu['single_core']['value']:.2f}/s on one ({cpu['cpu_model']})")

    import numpy as np
    import torch
    from paper_2112_06396_amd import hks, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    if args.w32_only:
        print(json.dumps(w32_extra(args, hks, synth, torch.cuda.current_stream())), flush=True)
        return
    if args.serving_only:
        print(json.dumps(serving_extra(args, hks, synth)), flush=True)
        return
    pq = hks.hks_gen_primes(50, LOG_N + 1, L + K)
    q, p = pq[:L], pq[L:]
    ctx = hks.Context(LOG_N, q, p, DNUM, max_batch=args.batch)
    n = 1 << LOG_N
    alpha = ctx.alpha
    beta = ctx.beta(LEVEL)
    key_mods = q + p
    # the main line runs the plan tuned for the plain Rotate (if cached)
    main_plan = contextlib.ExitStack()
    main_plan.enter_context(tuned_plan(hks, ctx, f"rotate_l{LEVEL}"))

    log(f"[bench] building pool of {args.pool} (ciphertext, key) pairs")
    cts, ksks, outs = [], [], []
    for i in range(args.pool):
        g = synth.rng(synth.seed_for(WORKLOAD, synth.KIND_CT, i))
        ct = np.stack([synth.uniform_residues(g, q[:LEVEL], n) for _ in range(2)])
        gk = synth.rng(synth.seed_for(WORKLOAD, synth.KIND_KEY, i))
        kk = np.stack([np.stack([synth.uniform_residues(gk, key_mods, n) for _ in range(2)]) for _ in range(DNUM)])
        cts.append(hks.to_device(ct))
        ksks.append(hks.to_device(kk))
        outs.append(hks.empty((2, LEVEL, n)))
    torch.cuda.synchronize()
    pool_bytes = sum(t.numel() * 8 for t in cts + ksks + outs)
    log(f"[bench] pool resident: {pool_bytes / 2**30:.2f} GiB")
    gal = hks.hks_galois_for_rotation(1, LOG_N)
    stream = torch.cuda.current_stream()
    if args.batched_only:
        main_plan.close()
        print(json.dumps(extras(args, ctx, hks, synth, cts, ksks, outs, gal, key_mods, n, None, stream)), flush=True)
        return

    def step(i):
        j = i % args.pool
        hks.hks_rotate(ctx, cts[j], LEVEL, gal, ksks[j], outs[j], stream)

    # warmup
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    # per-kernel breakdown (untimed pass, all classes recorded)
    hks.hks_prof_enable(ctx, (1 << 9) - 1)
    nb = min(20, max(4, args.steps // 10))
    for i in range(nb):
        step(i)
    torch.cuda.synchronize()
    breakdown = {}
    for cls, name in enumerate(hks.HKS_K_NAMES):
        ms, cnt = hks.hks_prof_read(ctx, cls)
        if cnt:
            breakdown[name] = {"ms_per_step": ms / nb, "launches_per_step": cnt / nb}
    hks.hks_prof_enable(ctx, 0)
    dom_name = max(breakdown, key=lambda k: breakdown[k]["ms_per_step"])
    dom_cls = hks.HKS_K_NAMES.index(dom_name)
    tot = sum(v["ms_per_step"] for v in breakdown.values())
    for k_, v in sorted(breakdown.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"[bench]   {k_:14s} {v['ms_per_step'] * 1e3:8.1f} us/step  {v['launches_per_step']:.0f} launches"
            f"  ({100 * v['ms_per_step'] / tot:.0f}%)")
    log(f"[bench] dominant kernel class: {dom_name}")

    # timed region: events at its two ends, and the dominant kernel's event
    # pair around each of its launches, recorded by the library
    hks.hks_prof_enable(ctx, 1 << dom_cls)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step(i)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dom_ms, dom_launches = hks.hks_prof_read(ctx, dom_cls)
    hks.hks_prof_enable(ctx, 0)
    gpu_ms = ev0.elapsed_time(ev1)
    # per-step latencies in a pass of their own (an event after every step
    # costs about 3 us per step, so it stays out of the timed region)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record(stream)
    for i in range(args.steps):
        step(i)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    ms_per_step = gpu_ms / args.steps
    value = args.steps / (gpu_ms / 1e3)
    log(f"[bench] timed {args.steps} steps: {ms_per_step * 1e3:.1f} us/step, {value:.0f} ks/s "
        f"(host wall {wall * 1e6 / args.steps:.1f} us/step)")

    # roofline of the dominant kernel
    mm, byt = kernel_work(dom_cls, n, LEVEL, K, alpha, beta)
    launches_per_step = dom_launches / args.steps
    avg_launch_s = dom_ms / 1e3 / dom_launches
    per_launch_mm = mm / launches_per_step
    per_launch_bytes = byt / launches_per_step
    if dom_cls <= 4:
        achieved = per_launch_mm / avg_launch_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": MODMUL_PEAK / 1e12, "unit": "Tmodmul/s",
                "frac": achieved / (MODMUL_PEAK / 1e12)}
    else:
        achieved = per_launch_bytes / avg_launch_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS}
    roof["kernel"] = dom_name
    roof["timing"] = ("HIP event pairs the library records around each launch of the kernel on its launch "
                      "stream, summed over the timed steps")
    roof["avg_launch_us"] = avg_launch_s * 1e6
    roof["launches_per_step"] = launches_per_step
    roof["algorithmic_per_launch"] = {"modmul": per_launch_mm, "bytes": per_launch_bytes}
    tr = read_traffic(dom_name)
    roof["traffic"] = tr
    # the counted bytes (L2 misses, Infinity Cache hits included) over the same duration
    roof["traffic_GBps"] = tr / avg_launch_s / 1e9 if tr else None

    # compulsory HBM bytes of one Rotate: a, b, key (digits < beta, limbs [0,level) U P), output
    key_bytes = beta * 2 * (LEVEL + K) * n * 8
    comp_bytes = 2 * LEVEL * n * 8 + key_bytes + 2 * LEVEL * n * 8
    # the whole key-switch against both rooflines: max(bytes / HBM, modmul / ALU)
    step_mm = sum(kernel_work(c_, n, LEVEL, K, alpha, beta)[0] for c_ in range(len(hks.HKS_K_NAMES)))
    whole = {"modmul_per_step": step_mm, "Tmodmul_per_s": step_mm / (ms_per_step / 1e3) / 1e12,
             "derived_Tmodmul_peak": MODMUL_PEAK / 1e12,
             "alu_frac": step_mm / (ms_per_step / 1e3) / MODMUL_PEAK,
             "hbm_frac": comp_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS}
    # the measured modular-product rate of the chip (lazy Shoup chains at full
    # occupancy) as the second ALU reference
    mm_rate = hks.hks_modmul_rate(ctx, 1024, stream)
    whole["measured_Tmodmul_peak"] = mm_rate / 1e12
    whole["alu_frac_of_measured"] = step_mm / (ms_per_step / 1e3) / mm_rate
    # a plain device copy of 1 GiB as the measured bandwidth reference
    src_ = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
    dst_ = torch.empty_like(src_)
    dst_.copy_(src_)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst_.copy_(src_)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src_.numel() * 8 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src_, dst_
    if roof["unit"] == "GB/s":
        roof["frac_of_measured_copy"] = roof["achieved"] / copy_gbs
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "key-switch/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "Rotate (key-switch) N=2^16 L=24 K=8 dnum=3 level=24, one 96 MiB key, "
                               f"pool of {args.pool} (ciphertext, key) pairs",
                   "log_n": LOG_N, "L": L, "K": K, "dnum": DNUM, "level": LEVEL, "batch": 1},
        "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)),
        "latency_source": "a second pass of the same steps after the timed region, an event after every step",
        "hbm_compulsory_bytes_per_step": comp_bytes,
        "hbm_algorithmic_GBps": comp_bytes / (ms_per_step / 1e3) / 1e9,
        "roofline": roof,
        "whole_keyswitch": whole,
        "measured_copy_GBps": copy_gbs,
        "kernel_breakdown_us": {k_: v["ms_per_step"] * 1e3 for k_, v in breakdown.items()},
        "env": {"numpy": np.__version__, "torch": torch.__version__, "hip": torch.version.hip,
                "arch": torch.cuda.get_device_properties(0).gcnArchName, "nproc": os.cpu_count()},
    }

    if not args.no_extras:
        main_plan.close()
        result.update(extras(args, ctx, hks, synth, cts, ksks, outs, gal, key_mods, n, value, stream))
    main_plan.close()
    result["launch_plans"] = dict(PLANS_USED)

    if args.calib_copy_mib:
        nw = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nw, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB done")

    if cpu:
        result["cpu_baseline"] = cpu

    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
