"""Parity at the edges of the lazy-reduction bounds and at the served shapes.

Every comparison is exact equality of uint64 residues with the CPU oracle.

  - Extreme words: every ciphertext, key and plaintext word is q - 1 (the
    largest canonical residue), or 0, at N = 2^16, L = 24, K = 8, dnum = 3,
    through Rotate, HRotate, batched Rotate with stored and seeded keys,
    Mult + relinearization + Rescale, NewMult and PtMatVecMult.  The kernels
    keep forward butterfly outputs lazy (below 35q) and sum the digits'
    128-bit products without reduction (Sec. 2.2); all-(q - 1) operands
    push those sums to their largest values.
  - More than 16 digits: alpha = 1 (dnum = L = 20), so beta reaches 20 and the
    key-switch kernels fold their lazy sums after every 16 digits; both word
    sizes, random and all-(q - 1) words.
  - The served shapes: N = 2^15 and 2^16 at L = 35, K = 12, dnum = 3 with
    batch contexts of 16 (batched Rotate with seeded keys, batched Mult with
    stored and seeded keys), and a serving run of both ring degrees whose
    results are the same alone and in the mix.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2112_06396_amd import synth

pytestmark = pytest.mark.gpu

_CTX = {}


def H():
    from paper_2112_06396_amd import hks
    return hks


def _get(shape, max_batch=1, bits=50):
    hks = H()
    key = (shape, max_batch, bits)
    if key not in _CTX:
        log_n, L, K, dnum = shape
        pr = O.make_params(log_n, L, K, dnum, bits=bits)
        if bits == 50:
            ctx = hks.Context(log_n, pr.q, pr.p, dnum, max_batch=max_batch)
        else:
            ctx = hks.Context32(log_n, pr.q, pr.p, dnum)
        _CTX[key] = (pr, ctx)
    return _CTX[key]


@pytest.fixture(scope="module", autouse=True)
def _cleanup():
    yield
    torch.cuda.synchronize()
    for _, ctx in _CTX.values():
        ctx.close()
    _CTX.clear()


def dev(a):
    return H().to_device(a)


def host(t):
    torch.cuda.synchronize()
    return H().to_host(t)


def _fill(mods, n, fill):
    """one limb per modulus, every word q - 1 ('max') or 0 ('zero')"""
    return np.stack([np.full(n, (int(q) - 1) if fill == "max" else 0, dtype=np.uint64) for q in mods])


def _ct(pr, level, fill, seed=0):
    if fill == "rand":
        g = synth.rng(seed)
        return np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])
    return np.stack([_fill(pr.q[:level], pr.n, fill)] * 2)


def _ksk(pr, fill, seed=0):
    if fill == "rand":
        g = synth.rng(seed)
        return np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                         for _ in range(pr.dnum)])
    return np.stack([np.stack([_fill(pr.key_mods(), pr.n, fill)] * 2)] * pr.dnum)


CFG2 = (16, 24, 8, 3)


@pytest.mark.parametrize("fill", ["max", "zero"])
def test_extreme_words_rotate_and_hoisted_forms(fill):
    """All words q - 1 (or 0) through Rotate, HRotate and batched Rotate with
    stored and seeded keys (a seeded key's rows b_j all q - 1 or 0)."""
    hks = H()
    pr, ctx = _get(CFG2, max_batch=2)
    level = pr.L
    ct, ksk = _ct(pr, level, fill), _ksk(pr, fill)
    d_ct, d_ksk = dev(ct), dev(ksk)
    gals = [hks.hks_galois_for_rotation(1, pr.log_n), hks.hks_galois_conjugate(pr.log_n)]
    out = hks.empty((2, level, pr.n))
    for g in gals:
        print(f"[extremes] fill={fill} rotate g={g}", flush=True)
        hks.hks_rotate(ctx, d_ct, level, g, d_ksk, out)
        ref = O.rotate(pr, ct, level, g, ksk)
        if fill == "zero":
            assert not ref.any()
        assert np.array_equal(host(out), ref), g
    print(f"[extremes] fill={fill} hrotate", flush=True)
    outs = [hks.empty((2, level, pr.n)) for _ in gals]
    hks.hks_hrotate(ctx, d_ct, level, gals, [d_ksk, d_ksk], outs)
    for o, r in zip(outs, O.hrotate(pr, ct, level, gals, [ksk, ksk])):
        assert np.array_equal(host(o), r)
    print(f"[extremes] fill={fill} batch rotate (stored, seeded)", flush=True)
    hks.hks_batch_rotate(ctx, [d_ct, d_ct], level, gals, [d_ksk, d_ksk], outs)
    for o, g in zip(outs, gals):
        assert np.array_equal(host(o), O.rotate(pr, ct, level, g, ksk))
    seeds = [0xE0, (1 << 64) - 1]
    b_row = np.ascontiguousarray(ksk[:, 1])
    hks.hks_batch_rotate_seeded(ctx, [d_ct, d_ct], level, gals, seeds, [dev(b_row)] * 2, outs)
    for o, g, sd in zip(outs, gals, seeds):
        full = np.stack([O.expand_key_a(pr, sd), b_row], axis=1)
        assert np.array_equal(host(o), O.rotate(pr, ct, level, g, full)), sd


@pytest.mark.parametrize("fill", ["max", "zero"])
def test_extreme_words_mult_newmult_ptmatvec(fill):
    """All words q - 1 (or 0) through Mult + relinearization + Rescale,
    NewMult and PtMatVecMult (two rotations and the diagonal without one)."""
    hks = H()
    pr, ctx = _get(CFG2, max_batch=2)
    level = pr.L
    ct, rlk = _ct(pr, level, fill), _ksk(pr, fill)
    d_ct, d_rlk = dev(ct), dev(rlk)
    print(f"[extremes] fill={fill} mult_relin", flush=True)
    out = hks.empty((2, level - 1, pr.n))
    hks.hks_mult_relin(ctx, d_ct, d_ct, level, d_rlk, True, out)
    assert np.array_equal(host(out), O.mult_relin(pr, ct, ct, level, rlk, True))
    print(f"[extremes] fill={fill} new_mult", flush=True)
    hks.hks_new_mult(ctx, d_ct, d_ct, level, d_rlk, out)
    assert np.array_equal(host(out), O.new_mult(pr, ct, ct, level, rlk))
    print(f"[extremes] fill={fill} ptmatvec", flush=True)
    gals = [hks.hks_galois_for_rotation(3, pr.log_n), 1, hks.hks_galois_for_rotation(-2, pr.log_n)]
    pts = [_fill(pr.ext_mods(level), pr.n, fill)] * 3
    ksks = [rlk, None, rlk]
    mv = hks.empty((2, level, pr.n))
    hks.hks_ptmatvec(ctx, d_ct, level, gals, [None if k is None else d_rlk for k in ksks], [dev(p) for p in pts],
                     mv)
    assert np.array_equal(host(mv), O.ptmatvec(pr, ct, level, gals, ksks, pts))


# alpha = 1: beta up to 20 digits, past the fold after 16
MANY = (10, 20, 1, 20)


@pytest.mark.parametrize("fill", ["rand", "max"])
def test_more_than_16_digits(fill):
    hks = H()
    pr, ctx = _get(MANY, max_batch=2)
    assert pr.alpha == 1
    g1 = hks.hks_galois_for_rotation(1, pr.log_n)
    g2 = hks.hks_galois_for_rotation(-5, pr.log_n)
    ksk = _ksk(pr, fill, 1700)
    d_ksk = dev(ksk)
    for level in (20, 17, 16):
        print(f"[extremes] beta={pr.beta(level)} fill={fill}", flush=True)
        ct = _ct(pr, level, fill, 1710 + level)
        d_ct = dev(ct)
        out = hks.empty((2, level, pr.n))
        hks.hks_rotate(ctx, d_ct, level, g1, d_ksk, out)
        assert np.array_equal(host(out), O.rotate(pr, ct, level, g1, ksk)), level
        outs = [hks.empty((2, level, pr.n)) for _ in range(2)]
        hks.hks_hrotate(ctx, d_ct, level, [g1, g2], [d_ksk, d_ksk], outs)
        for o, r in zip(outs, O.hrotate(pr, ct, level, [g1, g2], [ksk, ksk])):
            assert np.array_equal(host(o), r), level
        b_row = np.ascontiguousarray(ksk[:, 1])
        hks.hks_batch_rotate_seeded(ctx, [d_ct, d_ct], level, [g1, g2], [5, 6], [dev(b_row)] * 2, outs)
        for o, g, sd in zip(outs, (g1, g2), (5, 6)):
            full = np.stack([O.expand_key_a(pr, sd), b_row], axis=1)
            assert np.array_equal(host(o), O.rotate(pr, ct, level, g, full)), level
        mo = hks.empty((2, level - 1, pr.n))
        hks.hks_mult_relin(ctx, d_ct, d_ct, level, d_ksk, True, mo)
        assert np.array_equal(host(mo), O.mult_relin(pr, ct, ct, level, ksk, True)), level


@pytest.mark.parametrize("fill", ["rand", "max"])
def test_more_than_16_digits_w32(fill):
    """The 32-bit-word key switch (30-bit primes) sums the digits' products
    exactly in 64 bits and folds after every 16 digits."""
    hks = H()
    pr, ctx = _get(MANY, bits=30)
    g1 = hks.hks_galois_for_rotation(1, pr.log_n)
    g2 = hks.hks_galois_conjugate(pr.log_n)
    ksk = _ksk(pr, fill, 1800)
    d_ksk = hks.to_device32(ksk)
    for level in (20, 17):
        print(f"[extremes] w32 beta={pr.beta(level)} fill={fill}", flush=True)
        ct = _ct(pr, level, fill, 1810 + level)
        d_ct = hks.to_device32(ct)
        out = hks.empty32((2, level, pr.n))
        hks.hks32_rotate(ctx, d_ct, level, g1, d_ksk, out)
        torch.cuda.synchronize()
        assert np.array_equal(hks.to_host32(out), O.rotate(pr, ct, level, g1, ksk)), level
        outs = [hks.empty32((2, level, pr.n)) for _ in range(2)]
        hks.hks32_hrotate(ctx, d_ct, level, [g1, g2], [d_ksk, d_ksk], outs)
        torch.cuda.synchronize()
        for o, r in zip(outs, O.hrotate(pr, ct, level, [g1, g2], [ksk, ksk])):
            assert np.array_equal(hks.to_host32(o), r), level


# ------------------------------------------------------------------ the served shapes


def _dev_rand_ct(pr, level, seed):
    return synth.device_residues([int(q) for q in pr.q[:level]], (2,), pr.n, seed)


@pytest.mark.parametrize("log_n", [15, 16])
def test_served_shapes_batched_calls_equal_oracle(log_n):
    """L = 35, K = 12, dnum = 3 with a batch context of 16: batched Rotate
    with seeded keys and batched Mult + Rescale with stored and seeded keys,
    at the top level and at a level with one short digit, equal the oracle."""
    hks = H()
    pr, ctx = _get((log_n, 35, 12, 3), max_batch=16)
    nb = 3 if log_n == 15 else 2
    for level in (35, 13):
        print(f"[extremes] served N=2^{log_n} level={level}", flush=True)
        cts = [_ct(pr, level, "rand", 1900 + 10 * level + i) for i in range(nb + 1)]
        d_cts = [dev(c) for c in cts]
        b_rows = [np.ascontiguousarray(_ksk(pr, "rand", 1950 + i)[:, 1]) for i in range(nb)]
        seeds = [0x5E4 + i for i in range(nb)]
        fulls = [np.stack([O.expand_key_a(pr, sd), b], axis=1) for sd, b in zip(seeds, b_rows)]
        d_b = [dev(b) for b in b_rows]
        gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in (1, -3, 7)[:nb]]
        outs = [hks.empty((2, level, pr.n)) for _ in range(nb)]
        hks.hks_batch_rotate_seeded(ctx, d_cts[:nb], level, gals, seeds, d_b, outs)
        for i in range(nb):
            assert np.array_equal(host(outs[i]), O.rotate(pr, cts[i], level, gals[i], fulls[i])), (level, i)
        mouts = [hks.empty((2, level - 1, pr.n)) for _ in range(nb)]
        hks.hks_batch_mult_relin_seeded(ctx, d_cts[:nb], d_cts[1:], level, seeds, d_b, True, mouts)
        for i in range(nb):
            ref = O.mult_relin(pr, cts[i], cts[i + 1], level, fulls[i], True)
            assert np.array_equal(host(mouts[i]), ref), (level, i)
        hks.hks_batch_mult_relin(ctx, d_cts[:nb], d_cts[1:], level, [dev(f) for f in fulls], True, mouts)
        for i in range(nb):
            ref = O.mult_relin(pr, cts[i], cts[i + 1], level, fulls[i], True)
            assert np.array_equal(host(mouts[i]), ref), (level, i)


def test_serving_at_the_served_shapes_same_alone_and_in_the_mix():
    """The serving loop at N = 2^15 and 2^16, L = 35, K = 12, dnum = 3,
    steps of up to 16 requests on two lanes, fewer output slots than
    requests (admission waits for slots) and a key budget that forces
    evictions: every result equals the one-at-a-time run bit for bit, and
    one request of each N and op equals the oracle."""
    import copy
    from paper_2112_06396_amd import serving
    hks = H()
    prs = {ln: O.make_params(ln, 35, 12, 3) for ln in (15, 16)}
    n_clients = 4
    reqs = serving.poisson_requests(32, rate=4e4, n_clients=n_clients, log_ns=(15, 16), levels=(3, 35), seed=11)
    level_set = (35, 20, 3)
    for r in reqs:
        r.level = level_set[r.rid % 3]
    host_keys, seeds, b_np = {}, {}, {}
    for c in range(n_clients):
        ln = 15 if c % 2 == 0 else 16
        pr = prs[ln]
        for j, kind in enumerate(("rot", "rlk")):
            kid = (c, kind, ln)
            seeds[kid] = 0x5EED00 + 2 * c + j
            b = synth.device_residues([int(v) for v in pr.key_mods()], (3,), pr.n, 2000 + 2 * c + j)
            torch.cuda.synchronize()
            b_np[kid] = hks.to_host(b)
            host_keys[kid] = b.cpu().pin_memory()
            del b
    inputs = {}
    for ln, pr in prs.items():
        for level in level_set:
            inputs[(ln, level)] = [_dev_rand_ct(pr, level, 2100 + 10 * level + i + ln) for i in range(2)]
    params = {ln: (pr.q, pr.p, 3) for ln, pr in prs.items()}
    slot_words = max(t.numel() for t in host_keys.values())
    ks = serving.KeyStore(host_keys, budget=5 * slot_words * 8)
    ex = serving.HksExecutor(params, lanes=2, max_batch=16, slots_per_n=6, keystore=ks, inputs=inputs, seeds=seeds)
    # output slots are reused by later requests: capture each step's outputs
    # when its completion is observed (before the loop frees the slots)
    captured = {}
    batches = {}
    submit, done = ex.submit, ex.done

    def submit_capture(lane, batch):
        h = submit(lane, batch)
        batches[id(h)] = (h, batch)
        return h

    def done_capture(h):
        if not done(h):
            return False
        _, batch = batches.pop(id(h))
        for r in batch:
            captured[r.rid] = hks.to_host(ex.out_view(r)).copy()
        return True

    ex.submit, ex.done = submit_capture, done_capture
    try:
        eng = serving.Engine(ex, lanes=2, max_batch=16)
        alone = copy.deepcopy(reqs)
        print("[extremes] serving mix", flush=True)
        eng.run(reqs)
        torch.cuda.synchronize()
        mix, captured = captured, {}
        assert sorted(mix) == list(range(32))
        assert max(r.slot for r in reqs) < 6
        assert ks.uploads > len(host_keys)  # keys were evicted and uploaded again
        assert max(sum(1 for x in reqs if x.start == r.start) for r in reqs) > 1  # steps held several requests
        print("[extremes] serving alone", flush=True)
        eng.run(alone, one_at_a_time=True)
        torch.cuda.synchronize()
        assert sorted(captured) == list(range(32))
        for rid, want in mix.items():
            assert np.array_equal(captured[rid], want), rid
        checked = set()
        for r in reqs:
            key = (r.log_n, r.op)
            if key in checked:
                continue
            checked.add(key)
            pr = prs[r.log_n]
            pool = inputs[(r.log_n, r.level)]
            a = hks.to_host(pool[r.rid % len(pool)])
            kind = "rot" if r.op == "rotate" else "rlk"
            kid = (r.client, kind, r.log_n)
            full = np.stack([O.expand_key_a(pr, seeds[kid]), b_np[kid]], axis=1)
            print(f"[extremes] serving oracle check N=2^{r.log_n} {r.op} level={r.level}", flush=True)
            if r.op == "rotate":
                ref = O.rotate(pr, a, r.level, pow(5, -r.k, 2 * pr.n), full)
            else:
                b = hks.to_host(pool[(r.rid + 1) % len(pool)])
                ref = O.mult_relin(pr, a, b, r.level, full, True)
            assert np.array_equal(mix[r.rid], ref), r
    finally:
        ex.close()
