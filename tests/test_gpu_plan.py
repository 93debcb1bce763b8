"""Launch plans (include/hks.h, hks_plan) change only how launches are laid
over the chip: under extreme plans (16 or 8 elements per thread in every
pass, one NewLimb target per block row or all in one, block orders on or
off, the NTT split one stage either way of the default, 8 or 32 columns per
column-pass block, 4 or 16 rows per row-pass block) Rotate, HRotate,
batched Rotate, Mult+relin and PtMatVecMult equal the oracle bit for bit at
small sizes and equal the default plan at full size."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2112_06396_amd import synth, tune

pytestmark = pytest.mark.gpu

A8 = tune.ALWAYS8
# n1 "lo" / "hi": one stage fewer / more in the column pass than the default
# split, where the ring degree allows it (_resolve)
PLANS = {
    "e16_all_split": {"e16_fwd_cols": 0, "e16_fwd_rows": 0, "e16_inv_rows": 0, "e16_inv_cols": 0,
                      "conv_group_limbs": 1, "conv_group_max_batch": 64, "row_xcd_order": 0, "ksk_xcd_order": 0,
                      "n1": "lo", "col_lines": 32, "row_lines": 16},
    "e8_all_whole": {"e16_fwd_cols": A8, "e16_fwd_rows": A8, "e16_inv_rows": A8, "e16_inv_cols": A8,
                     "conv_group_limbs": 64, "conv_group_max_batch": 0, "row_xcd_order": 1, "ksk_xcd_order": 1,
                     "n1": "hi", "col_lines": 8, "row_lines": 4},
    "mixed": {"e16_fwd_cols": 0, "e16_fwd_rows": A8, "e16_inv_rows": 0, "e16_inv_cols": A8,
              "conv_group_limbs": 4, "conv_group_max_batch": 1, "row_xcd_order": 1, "ksk_xcd_order": 0,
              "n1": 0, "col_lines": 16, "row_lines": 8},
}


def _resolve(plan, log_n):
    p = dict(plan)
    if p["n1"] in ("lo", "hi"):
        h = log_n // 2
        want = h - 1 if p["n1"] == "lo" else h + 1
        p["n1"] = want if want in tune.candidates_for(log_n)["n1"] else 0
    return p
CFGS = {"n10": (10, 6, 2, 3), "n13": (13, 7, 3, 3), "n15": (15, 6, 2, 3)}
_CTX = {}


def H():
    from paper_2112_06396_amd import hks
    return hks


def _get(cfg, max_batch=4):
    key = (cfg, max_batch)
    if key not in _CTX:
        log_n, L, K, dnum = CFGS[cfg] if cfg in CFGS else cfg
        pr = O.make_params(log_n, L, K, dnum)
        _CTX[key] = (pr, H().Context(log_n, pr.q, pr.p, dnum, max_batch=max_batch))
    return _CTX[key]


@pytest.fixture(scope="module", autouse=True)
def _cleanup():
    yield
    torch.cuda.synchronize()
    for _, ctx in _CTX.values():
        ctx.close()
    _CTX.clear()


def host(t):
    torch.cuda.synchronize()
    return H().to_host(t)


def _ct(pr, level, seed):
    g = synth.rng(seed)
    return np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])


def _ksk(pr, seed):
    g = synth.rng(seed)
    return np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                     for _ in range(pr.dnum)])


def test_plan_get_set_and_rejection():
    hks = H()
    pr, ctx = _get("n10")
    d = hks.hks_get_plan(ctx)
    assert d == {"e16_fwd_cols": 6144, "e16_fwd_rows": A8, "e16_inv_rows": 6144, "e16_inv_cols": 6144,
                 "conv_group_limbs": 8, "conv_group_max_batch": 2, "row_xcd_order": 1, "ksk_xcd_order": 1,
                 "n1": 0, "col_lines": 16, "row_lines": 8}
    hks.hks_set_plan(ctx, PLANS["mixed"])
    assert hks.hks_get_plan(ctx) == PLANS["mixed"]
    # N = 2^10 allows only the 5 x 5 split
    for bad in ({"conv_group_limbs": 0}, {"conv_group_limbs": 65}, {"row_xcd_order": 2}, {"ksk_xcd_order": 7},
                {"col_lines": 12}, {"row_lines": 32}, {"n1": 4}, {"n1": 6}):
        with pytest.raises(hks.HksError) as e:
            hks.hks_set_plan(ctx, bad)
        assert e.value.status == hks.HKS_EINVAL
        assert hks.hks_get_plan(ctx) == PLANS["mixed"]
    hks.hks_set_plan(ctx, d)


@pytest.mark.parametrize("plan", list(PLANS))
@pytest.mark.parametrize("cfg", list(CFGS))
def test_calls_equal_oracle_under_plan(cfg, plan):
    hks = H()
    pr, ctx = _get(cfg)
    default = hks.hks_get_plan(ctx)
    hks.hks_set_plan(ctx, _resolve(PLANS[plan], pr.log_n))
    try:
        level = pr.L
        ct = _ct(pr, level, 900)
        ksks = [_ksk(pr, 901 + i) for i in range(3)]
        dks = [hks.to_device(k) for k in ksks]
        gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in (1, -2, 5)]
        dct = hks.to_device(ct)
        # Rotate
        out = hks.empty((2, level, pr.n))
        hks.hks_rotate(ctx, dct, level, gals[0], dks[0], out)
        assert np.array_equal(host(out), O.rotate(pr, ct, level, gals[0], ksks[0]))
        # HRotate (3 rotations, steps of the context's batch capacity)
        outs = [hks.empty((2, level, pr.n)) for _ in gals]
        hks.hks_hrotate(ctx, dct, level, gals, dks, outs)
        for o, w in zip(outs, O.hrotate(pr, ct, level, gals, ksks)):
            assert np.array_equal(host(o), w)
        # batched Rotate of 3 ciphertexts with their own keys, one level below the top
        lv = level - 1
        cts = [_ct(pr, lv, 910 + i) for i in range(3)]
        outs = [hks.empty((2, lv, pr.n)) for _ in cts]
        hks.hks_batch_rotate(ctx, [hks.to_device(c) for c in cts], lv, gals, dks, outs)
        for c, g, k, o in zip(cts, gals, ksks, outs):
            assert np.array_equal(host(o), O.rotate(pr, c, lv, g, k))
        # Mult + relinearization + Rescale
        ct2 = _ct(pr, level, 920)
        mo = hks.empty((2, level - 1, pr.n))
        hks.hks_mult_relin(ctx, dct, hks.to_device(ct2), level, dks[1], True, mo)
        assert np.array_equal(host(mo), O.mult_relin(pr, ct, ct2, level, ksks[1], True))
        # PtMatVecMult over two rotations and the diagonal without rotation
        g = synth.rng(930)
        pts = [synth.uniform_residues(g, list(pr.q[:level]) + list(pr.p), pr.n) for _ in range(3)]
        mv = hks.empty((2, level, pr.n))
        hks.hks_ptmatvec(ctx, dct, level, [gals[0], gals[1], 1], [dks[0], dks[1], None],
                         [hks.to_device(p) for p in pts], mv)
        assert np.array_equal(host(mv), O.ptmatvec(pr, ct, level, [gals[0], gals[1], 1],
                                                   [ksks[0], ksks[1], None], pts))
    finally:
        hks.hks_set_plan(ctx, default)


def test_full_size_plans_equal_default():
    """N = 2^16, L = 24, K = 8, dnum = 3: Rotate, batched Rotate (16 per
    step) and HRotate give the same words under every plan."""
    hks = H()
    pq = hks.hks_gen_primes(50, 17, 32)
    ctx = hks.Context(16, pq[:24], pq[24:], 3, max_batch=16)
    try:
        n = 1 << 16
        cts = [synth.device_residues(pq[:24], (2,), n, 940 + i) for i in range(16)]
        keys = [synth.device_residues(pq, (3, 2), n, 960 + i) for i in range(16)]
        gals = [hks.hks_galois_for_rotation(k + 1, 16) for k in range(16)]

        def run_all():
            o1 = hks.empty((2, 24, n))
            hks.hks_rotate(ctx, cts[0], 24, gals[0], keys[0], o1)
            ob = [hks.empty((2, 24, n)) for _ in range(16)]
            hks.hks_batch_rotate(ctx, cts, 24, gals, keys, ob)
            oh = [hks.empty((2, 24, n)) for _ in range(16)]
            hks.hks_hrotate(ctx, cts[1], 24, gals, keys, oh)
            torch.cuda.synchronize()
            return [o1] + ob + oh

        ref = [t.view(torch.int64).clone() for t in run_all()]
        for name, plan in PLANS.items():
            hks.hks_set_plan(ctx, _resolve(plan, 16))
            got = run_all()
            assert all(torch.equal(a, b.view(torch.int64)) for a, b in zip(ref, got)), name
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_tuner_end_to_end_small():
    """tune.tune on a small Rotate workload: times every candidate of two
    fields, keeps a plan whose outputs equal the start plan's, and returns a
    cache entry that apply_cached restores."""
    import json
    import os
    import tempfile
    hks = H()
    pr, ctx = _get("n13")
    level = pr.L
    ct = hks.to_device(_ct(pr, level, 990))
    key = hks.to_device(_ksk(pr, 991))
    out = hks.empty((2, level, pr.n))
    gal = hks.hks_galois_for_rotation(3, pr.log_n)
    stream = torch.cuda.current_stream()
    start = hks.hks_get_plan(ctx)

    def run(i):
        hks.hks_rotate(ctx, ct, level, gal, key, out, stream)

    cands = {"conv_group_limbs": (4, 8, 16), "e16_fwd_cols": (0, A8)}
    best, t_best, t_start, trace = tune.coordinate_descent(tune.event_measure(ctx, run, stream, 5), start,
                                                           candidates=cands, rounds=1)
    # one pass: every candidate value other than the incumbent's is timed (a
    # value kept part-way makes the start value a candidate again)
    assert 1 + sum(len([v for v in vals if v != start[f]]) for f, vals in cands.items()) <= len(trace)
    assert len(trace) <= 1 + sum(len(vals) for vals in cands.values())
    assert t_best <= t_start
    hks.hks_set_plan(ctx, start)
    entry = tune.tune(ctx, run, lambda: [out], stream, 5, rounds=1)
    assert entry["outputs_equal"] and entry["us"] <= entry["default_us"] and set(entry["plan"]) == set(start)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "plans.json")
        tune.save_entry("k", entry, path)
        hks.hks_set_plan(ctx, start)
        assert tune.apply_cached(ctx, "k", path)["plan"] == entry["plan"]
        assert hks.hks_get_plan(ctx) == entry["plan"]
        assert tune.apply_cached(ctx, "missing", path) is None
        with open(path) as f:
            json.load(f)
    hks.hks_set_plan(ctx, start)
    torch.cuda.synchronize()
    assert np.array_equal(host(out), O.rotate(pr, _ct(pr, level, 990), level, gal, _ksk(pr, 991)))
