"""Parity of the HIP path with the CPU oracle, through the C ABI.

Every comparison is exact equality of uint64 residues (the method is exact
modular arithmetic; both sides reduce to canonical [0, q)).  Inputs are
seeded synthetic residues from paper_2112_06396_amd.synth; valid keys and
ciphertexts (for the decryption checks) come from the oracle's test-side
key generation.  Shapes cover several NTT tiles and splits (log N = 10..16,
odd sub-transform sizes), short last digits, level 1, more special primes
than a digit has limbs (K = 4 > alpha = 3 at N = 2^14), and the full
N = 2^16, L = 24, K = 8, dnum = 3 key-switch and L = 35, K = 12.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2112_06396_amd import synth

pytestmark = pytest.mark.gpu

CFGS = {
    # name: (log_n, L, K, dnum)
    "n10": (10, 6, 2, 3),
    "n11": (11, 5, 3, 2),
    "cfg1": (12, 4, 2, 2),
    "n13": (13, 7, 3, 3),
    "n14": (14, 9, 4, 3),
    "n15": (15, 6, 2, 3),
    "cfg2": (16, 24, 8, 3),
}

_CTX = {}


def _get(name, max_batch=1):
    from paper_2112_06396_amd import hks
    key = (name, max_batch)
    if key not in _CTX:
        log_n, L, K, dnum = CFGS[name] if name in CFGS else name
        pr = O.make_params(log_n, L, K, dnum)
        _CTX[key] = (pr, hks.Context(log_n, pr.q, pr.p, dnum, max_batch=max_batch))
    return _CTX[key]


@pytest.fixture(scope="module", autouse=True)
def _cleanup():
    yield
    for _, ctx in _CTX.values():
        ctx.close()
    _CTX.clear()


def H():
    from paper_2112_06396_amd import hks
    return hks


def dev(a):
    return H().to_device(a)


def host(t):
    torch.cuda.synchronize()
    return H().to_host(t)


def _rand_ct(pr, level, seed):
    g = synth.rng(seed)
    return np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])


def _rand_ksk(pr, seed):
    g = synth.rng(seed)
    return np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                     for _ in range(pr.dnum)])


def _levels(pr):
    return sorted({1, pr.alpha + 1, pr.L - 1, pr.L} - {0})


# ------------------------------------------------------------------ NTT / automorph

@pytest.mark.parametrize("name", list(CFGS))
def test_ntt_intt(name):
    pr, ctx = _get(name)
    hks = H()
    mods = pr.key_mods()
    x = synth.uniform_residues(synth.rng(10), mods, pr.n)
    d = dev(x)
    hks.hks_ntt(ctx, d, 0, len(mods))
    y = host(d)
    assert np.array_equal(y, O.ntt(x, pr.log_n, mods))
    hks.hks_intt(ctx, d, 0, len(mods))
    assert np.array_equal(host(d), x)
    # a sub-range of moduli (the special primes)
    z = synth.uniform_residues(synth.rng(11), pr.p, pr.n)
    dz = dev(z)
    hks.hks_intt(ctx, dz, pr.L, pr.K)
    assert np.array_equal(host(dz), O.intt(z, pr.log_n, pr.p))


@pytest.mark.parametrize("name", ["n10", "cfg1", "cfg2"])
def test_automorph_eval_and_coeff(name):
    pr, ctx = _get(name)
    hks = H()
    x = synth.uniform_residues(synth.rng(12), pr.q, pr.n)
    d = dev(x)
    out = hks.empty(x.shape)
    for g in (hks.hks_galois_for_rotation(1, pr.log_n), hks.hks_galois_for_rotation(-7, pr.log_n),
              hks.hks_galois_conjugate(pr.log_n)):
        for ev in (True, False):
            hks.hks_automorph(ctx, d, out, 0, pr.L, g, ev)
            assert np.array_equal(host(out), O.automorph(x, pr.log_n, pr.q, g, eval_domain=ev))


# ------------------------------------------------------------------ subroutines

@pytest.mark.parametrize("name", ["n10", "n11", "cfg1", "n13", "cfg2"])
def test_modup(name):
    pr, ctx = _get(name)
    hks = H()
    for level in _levels(pr):
        a = synth.uniform_residues(synth.rng(20 + level), pr.q[:level], pr.n)
        ext = hks.empty((pr.beta(level), level + pr.K, pr.n))
        hks.hks_modup(ctx, dev(a), level, ext)
        assert np.array_equal(host(ext), O.modup(pr, a, level)), level


@pytest.mark.parametrize("name", ["n10", "cfg1", "cfg2"])
def test_ksk_inner(name):
    pr, ctx = _get(name)
    hks = H()
    ksk = _rand_ksk(pr, 30)
    dk = dev(ksk)
    for level in _levels(pr):
        g = synth.rng(31 + level)
        ext = np.stack([synth.uniform_residues(g, pr.ext_mods(level), pr.n) for _ in range(pr.beta(level))])
        uv = hks.empty((2, level + pr.K, pr.n))
        hks.hks_ksk_inner(ctx, dev(ext), level, dk, uv)
        assert np.array_equal(host(uv), O.ksk_inner(pr, ext, level, ksk)), level


@pytest.mark.parametrize("name", ["n10", "n11", "cfg1", "n15", "cfg2"])
def test_moddown(name):
    pr, ctx = _get(name)
    hks = H()
    for level in _levels(pr):
        x = synth.uniform_residues(synth.rng(40 + level), pr.ext_mods(level), pr.n)
        y = hks.empty((level, pr.n))
        hks.hks_moddown(ctx, dev(x), level, y)
        assert np.array_equal(host(y), O.moddown(pr, x, level)), level


# ------------------------------------------------------------------ composite calls

@pytest.mark.parametrize("name", ["n10", "n11", "cfg1", "n13", "n14", "n15", "cfg2"])
def test_keyswitch(name):
    pr, ctx = _get(name)
    hks = H()
    ksk = _rand_ksk(pr, 50)
    dk = dev(ksk)
    for level in _levels(pr):
        d = synth.uniform_residues(synth.rng(51 + level), pr.q[:level], pr.n)
        uv = hks.empty((2, level, pr.n))
        hks.hks_keyswitch(ctx, dev(d), level, dk, uv)
        assert np.array_equal(host(uv), O.keyswitch(pr, d, level, ksk)), level


@pytest.mark.parametrize("name", ["n10", "n11", "cfg1", "n13", "n14", "n15", "cfg2"])
def test_rotate(name):
    pr, ctx = _get(name)
    hks = H()
    ksk = _rand_ksk(pr, 60)
    dk = dev(ksk)
    for level in _levels(pr):
        # rotations by 1 and -3 and the conjugation (galois 2N - 1)
        for g in (hks.hks_galois_for_rotation(1, pr.log_n), hks.hks_galois_for_rotation(-3, pr.log_n),
                  hks.hks_galois_conjugate(pr.log_n)):
            ct = _rand_ct(pr, level, 61 + level)
            out = hks.empty((2, level, pr.n))
            hks.hks_rotate(ctx, dev(ct), level, g, dk, out)
            assert np.array_equal(host(out), O.rotate(pr, ct, level, g, ksk)), (level, g)


def test_rotate_config1_valid_key_decrypts():
    """config 1: N=2^12, 4 limbs, 2 special primes, dnum=2, ternary secret,
    rotation index 1; GPU output equals the oracle and decrypts to the
    rotated message within the key-switching noise bound."""
    pr, ctx = _get("cfg1")
    hks = H()
    g = synth.rng(synth.seed_for(1, synth.KIND_SECRET))
    s = synth.ternary(g, pr.n)
    gal = hks.hks_galois_for_rotation(1, pr.log_n)
    ksk = O.rotation_key(pr, s, gal, g)
    ct = O.encrypt(pr, s, synth.small_uniform(g, pr.n, 1 << 40), 4, g)
    out = hks.empty((2, 4, pr.n))
    hks.hks_rotate(ctx, dev(ct), 4, gal, dev(ksk), out)
    got = host(out)
    assert np.array_equal(got, O.rotate(pr, ct, 4, gal, ksk))
    mods = pr.q[:4]
    diff = O.sub_vec(O.decrypt_coef(pr, s, got, 4),
                     O.automorph(O.decrypt_coef(pr, s, ct, 4), pr.log_n, mods, gal, eval_domain=False),
                     pr.log_n, mods)
    assert O.centered_small(diff, mods, O.ks_noise_bound(pr, 4, s)) is not None


def test_rotate_config2_valid_key_decrypts():
    """N=2^16, L=24, K=8, dnum=3 with a valid rotation key: bit-exact vs the
    oracle and decryption within the noise bound."""
    pr, ctx = _get("cfg2")
    hks = H()
    g = synth.rng(synth.seed_for(2, synth.KIND_SECRET))
    s = synth.ternary(g, pr.n)
    gal = hks.hks_galois_for_rotation(1, pr.log_n)
    ksk = O.rotation_key(pr, s, gal, g)
    level = 24
    ct = O.encrypt(pr, s, synth.small_uniform(g, pr.n, 1 << 40), level, g)
    out = hks.empty((2, level, pr.n))
    hks.hks_rotate(ctx, dev(ct), level, gal, dev(ksk), out)
    got = host(out)
    assert np.array_equal(got, O.rotate(pr, ct, level, gal, ksk))
    mods = pr.q[:level]
    diff = O.sub_vec(O.decrypt_coef(pr, s, got, level),
                     O.automorph(O.decrypt_coef(pr, s, ct, level), pr.log_n, mods, gal, eval_domain=False),
                     pr.log_n, mods)
    assert O.centered_small(diff, mods, O.ks_noise_bound(pr, level, s)) is not None


@pytest.mark.parametrize("name", ["n10", "cfg1", "cfg2"])
def test_hrotate(name):
    pr, ctx = _get(name)
    hks = H()
    level = pr.L
    # three rotations and the conjugation
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in (1, 2, -5)] + [hks.hks_galois_conjugate(pr.log_n)]
    ksks = [_rand_ksk(pr, 70 + i) for i in range(len(gals))]
    ct = _rand_ct(pr, level, 75)
    outs = [hks.empty((2, level, pr.n)) for _ in gals]
    hks.hks_hrotate(ctx, dev(ct), level, gals, [dev(k) for k in ksks], outs)
    refs = O.hrotate(pr, ct, level, gals, ksks)
    for o, r in zip(outs, refs):
        assert np.array_equal(host(o), r)


@pytest.mark.parametrize("name,max_batch,r", [("n10", 2, 5), ("cfg1", 4, 3), ("cfg2", 4, 6)])
def test_hrotate_batched_steps(name, max_batch, r):
    """Rotations processed max_batch at a time (ragged last step) equal the
    oracle's HRotate (Algorithm 4) exactly."""
    pr, ctx = _get(name, max_batch)
    hks = H()
    level = pr.L - 1 if pr.L > 1 else pr.L
    ks = [1, -1, 3, 7, -16, 2][:r]
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in ks]
    ksks = [_rand_ksk(pr, 120 + i) for i in range(r)]
    ct = _rand_ct(pr, level, 126)
    outs = [hks.empty((2, level, pr.n)) for _ in ks]
    hks.hks_hrotate(ctx, dev(ct), level, gals, [dev(k) for k in ksks], outs)
    refs = O.hrotate(pr, ct, level, gals, ksks)
    for i, (o, ref) in enumerate(zip(outs, refs)):
        assert np.array_equal(host(o), ref), i


@pytest.mark.parametrize("name,max_batch,n_ct,shared", [
    ("n10", 4, 6, False), ("cfg1", 8, 8, True), ("cfg1", 3, 7, False), ("n13", 16, 5, True),
    ("cfg2", 8, 8, True), ("cfg2", 4, 5, False)])
def test_batch_rotate_batched_context(name, max_batch, n_ct, shared):
    """Batched Rotate with a shared key (one galois) or distinct keys and
    galois elements, in steps of max_batch (ragged last step): every output
    equals the oracle's Rotate of that ciphertext (Algorithm 3)."""
    pr, ctx = _get(name, max_batch)
    hks = H()
    level = pr.L
    nk = 1 if shared else n_ct
    ksks = [_rand_ksk(pr, 130 + i) for i in range(nk)]
    dks = [dev(k) for k in ksks]
    ks = [1] * n_ct if shared else [1 + (3 * i) % 11 - 5 for i in range(n_ct)]
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in ks]
    cts = [_rand_ct(pr, level, 140 + i) for i in range(n_ct)]
    outs = [hks.empty((2, level, pr.n)) for _ in cts]
    kidx = [0 if shared else i for i in range(n_ct)]
    hks.hks_batch_rotate(ctx, [dev(c) for c in cts], level, gals, [dks[j] for j in kidx], outs)
    for i in range(n_ct):
        ref = O.rotate(pr, cts[i], level, gals[i], ksks[kidx[i]])
        assert np.array_equal(host(outs[i]), ref), i


def test_batched_context_single_calls_and_lower_level():
    """A context with batch slots still gives the single-call results, and a
    batch at a lower level (short last digit) after a full-level batch."""
    pr, ctx = _get("n13", 4)
    hks = H()
    ksk = _rand_ksk(pr, 150)
    dk = dev(ksk)
    c1, c2 = _rand_ct(pr, pr.L, 151), _rand_ct(pr, pr.L, 152)
    o = hks.empty((2, pr.L, pr.n))
    hks.hks_mult_relin(ctx, dev(c1), dev(c2), pr.L, dk, False, o)
    assert np.array_equal(host(o), O.mult_relin(pr, c1, c2, pr.L, ksk, False))
    uv = hks.empty((2, pr.L, pr.n))
    hks.hks_keyswitch(ctx, dev(c1[0]), pr.L, dk, uv)
    assert np.array_equal(host(uv), O.keyswitch(pr, c1[0], pr.L, ksk))
    level = pr.alpha + 1
    g = hks.hks_galois_for_rotation(2, pr.log_n)
    cts = [_rand_ct(pr, level, 153 + i) for i in range(3)]
    outs = [hks.empty((2, level, pr.n)) for _ in cts]
    hks.hks_batch_rotate(ctx, [dev(c) for c in cts], level, [g] * 3, [dk] * 3, outs)
    for c, out in zip(cts, outs):
        assert np.array_equal(host(out), O.rotate(pr, c, level, g, ksk))


def test_batch_rotate_rejects_aliasing():
    pr, ctx = _get("cfg1", 4)
    hks = H()
    cts = [dev(_rand_ct(pr, 4, 160 + i)) for i in range(2)]
    ksk = dev(_rand_ksk(pr, 162))
    out = hks.empty((2, 4, pr.n))
    with pytest.raises(hks.HksError):
        hks.hks_batch_rotate(ctx, cts, 4, [5, 5], [ksk, ksk], [out, cts[0]])
    with pytest.raises(hks.HksError):
        hks.hks_batch_rotate(ctx, cts, 4, [5, 5], [ksk, ksk], [out, out])


@pytest.mark.parametrize("name", ["cfg1", "cfg2"])
def test_batch_rotate_equals_single(name):
    pr, ctx = _get(name)
    hks = H()
    level = pr.L
    ksk = _rand_ksk(pr, 80)
    dk = dev(ksk)
    cts = [_rand_ct(pr, level, 81 + i) for i in range(3)]
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in (1, 1, 4)]
    outs = [hks.empty((2, level, pr.n)) for _ in cts]
    hks.hks_batch_rotate(ctx, [dev(c) for c in cts], level, gals, [dk] * 3, outs)
    for c, gl, o in zip(cts, gals, outs):
        assert np.array_equal(host(o), O.rotate(pr, c, level, gl, ksk))


@pytest.mark.parametrize("name", ["n10", "cfg1", "cfg2"])
def test_rescale_ptmult(name):
    pr, ctx = _get(name)
    hks = H()
    for level in sorted({2, pr.L}):
        ct = _rand_ct(pr, level, 90 + level)
        pt = synth.uniform_residues(synth.rng(91), pr.q[:level], pr.n)
        out = hks.empty((2, level - 1, pr.n))
        hks.hks_rescale(ctx, dev(ct), level, out)
        assert np.array_equal(host(out), O.rescale(pr, ct, level))
        for rs in (False, True):
            o = hks.empty((2, level - (1 if rs else 0), pr.n))
            hks.hks_ptmult(ctx, dev(ct), dev(pt), level, rs, o)
            assert np.array_equal(host(o), O.ptmult(pr, ct, pt, level, rs))


@pytest.mark.parametrize("name", ["n10", "cfg1", "cfg2"])
def test_mult_relin(name):
    pr, ctx = _get(name)
    hks = H()
    rlk = _rand_ksk(pr, 100)
    level = pr.L
    c1, c2 = _rand_ct(pr, level, 101), _rand_ct(pr, level, 102)
    for rs in (False, True):
        o = hks.empty((2, level - (1 if rs else 0), pr.n))
        hks.hks_mult_relin(ctx, dev(c1), dev(c2), level, dev(rlk), rs, o)
        assert np.array_equal(host(o), O.mult_relin(pr, c1, c2, level, rlk, rs))


def test_max_level_config4_shape():
    """N=2^16 at the top of the bootstrapping-shaped trace: L=35, K=12, dnum=3."""
    pr, ctx = _get((16, 35, 12, 3))
    hks = H()
    ksk = _rand_ksk(pr, 110)
    for level in (35, 10):
        ct = _rand_ct(pr, level, 111)
        g = hks.hks_galois_for_rotation(32, pr.log_n)
        out = hks.empty((2, level, pr.n))
        hks.hks_rotate(ctx, dev(ct), level, g, dev(ksk), out)
        assert np.array_equal(host(out), O.rotate(pr, ct, level, g, ksk)), level


def test_invalid_arguments_are_rejected():
    pr, ctx = _get("cfg1")
    hks = H()
    ct = dev(_rand_ct(pr, 4, 1))
    ksk = dev(_rand_ksk(pr, 2))
    out = hks.empty((2, 4, pr.n))
    for level, g in ((0, 5), (5, 5), (4, 4), (4, 2 * pr.n + 1)):
        with pytest.raises(hks.HksError) as e:
            hks.hks_rotate(ctx, ct, level, g, ksk, out)
        assert e.value.status == hks.HKS_EINVAL
    with pytest.raises(hks.HksError):
        hks.hks_rotate(ctx, ct, 4, 5, ksk, ct)  # output aliases input
    with pytest.raises(hks.HksError):
        hks.hks_rescale(ctx, ct, 1, out)


def test_deterministic_repeat():
    pr, ctx = _get("cfg2")
    hks = H()
    ct, ksk = dev(_rand_ct(pr, 24, 5)), dev(_rand_ksk(pr, 6))
    o1, o2 = hks.empty((2, 24, pr.n)), hks.empty((2, 24, pr.n))
    g = hks.hks_galois_for_rotation(1, pr.log_n)
    hks.hks_rotate(ctx, ct, 24, g, ksk, o1)
    hks.hks_rotate(ctx, ct, 24, g, ksk, o2)
    assert torch.equal(o1.view(torch.int64), o2.view(torch.int64))


# ------------------------------------------------------------------ bootstrapping-shaped trace, hipGraph


def _oracle_plan(pr, plan, x0, diag, keys, rlk):
    """The plan's ops through the oracle (Algorithms 1, 2, 4 and Rescale)."""
    bufs = {"x0": x0}
    for op in plan.ops:
        kind = op[0]
        if kind == "hrotate":
            _, src, level, ks, dsts = op
            gals = [pow(5, -k, 2 * pr.n) for k in ks]
            outs = O.hrotate(pr, bufs[src], level, gals, [keys[k] for k in ks])
            for d, o in zip(dsts, outs):
                bufs[d] = o
        elif kind == "ptmult":
            _, src, d, level, dst = op
            bufs[dst] = O.ptmult(pr, bufs[src], diag[d][:level], level, False)
        elif kind == "ptmatvec":
            _, src, level, ks, ds, dst = op
            gals = [pow(5, -k, 2 * pr.n) if k else 1 for k in ks]
            pts = [np.concatenate([diag[d][:level], diag[d][pr.L:]]) for d in ds]
            bufs[dst] = O.ptmatvec(pr, bufs[src], level, gals, [keys[k] if k else None for k in ks], pts)
        elif kind == "add":
            _, a, b, level, dst = op
            bufs[dst] = np.stack([O.add_vec(bufs[a][i], bufs[b][i], pr.log_n, pr.q[:level]) for i in range(2)])
        elif kind == "rescale":
            _, src, level, dst = op
            bufs[dst] = O.rescale(pr, bufs[src], level)
        elif kind == "mult":
            _, a, b, level, dst = op
            bufs[dst] = O.mult_relin(pr, bufs[a], bufs[b], level, rlk, True)
        elif kind == "newmult":
            _, a, b, level, dst = op
            bufs[dst] = O.new_mult(pr, bufs[a], bufs[b], level, rlk)
        elif kind in ("mults", "newmults"):
            _, prods, level = op
            res = [O.mult_relin(pr, bufs[a], bufs[b], level, rlk, True) if kind == "mults"
                   else O.new_mult(pr, bufs[a], bufs[b], level, rlk) for a, b, _ in prods]
            for (_, _, d), r in zip(prods, res):
                bufs[d] = r
    return bufs[plan.out]


def test_trace_eager_and_graph_replays_match_oracle():
    """A small bootstrapping-shaped trace (hoisted stages, PtMult sums,
    Rescale, Mult + relin at falling levels, mirrored stages) run eagerly and
    as one captured hipGraph replayed three times, with eager library work
    and buffer clearing between replays: every result equals the oracle's."""
    from paper_2112_06396_amd import trace
    pr, ctx = _get((12, 10, 4, 3), 4)
    hks = H()
    plan = trace.bootstrap_plan(pr.L, counts=(2, 2, 3), strides=(1, 4, 16), evalmod_levels=3)
    g = synth.rng(200)
    x0 = _rand_ct(pr, pr.L, 201)
    diag = {d: synth.uniform_residues(g, pr.q, pr.n) for d in plan.diagonals}
    keys = {k: _rand_ksk(pr, 300 + i) for i, k in enumerate(plan.rotations)}
    rlk = _rand_ksk(pr, 299)
    ref = _oracle_plan(pr, plan, x0, diag, keys, rlk)

    bufs = trace.TraceBuffers(plan, pr.n)
    bufs.view("x0", pr.L).copy_(dev(x0))
    ddiag = {d: dev(v) for d, v in diag.items()}
    dkeys = {k: dev(v) for k, v in keys.items()}
    drlk = dev(rlk)
    out = trace.run_plan(ctx, plan, bufs, ddiag, dkeys, drlk)
    assert np.array_equal(host(out), ref)

    gr = trace.capture(ctx, plan, bufs, ddiag, dkeys, drlk)
    other = dev(_rand_ct(pr, pr.L, 202))
    other_out = hks.empty((2, pr.L, pr.n))
    for rep in range(3):
        for name, t in bufs.ct.items():
            if name != "x0":
                t.zero_()
        hks.hks_rotate(ctx, other, pr.L, hks.hks_galois_for_rotation(3, pr.log_n), dkeys[plan.rotations[0]],
                       other_out)
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(bufs.view(plan.out, plan.out_level)), ref), rep


def test_hoisted_trace_eager_and_graph_match_oracle():
    """The same small trace with every linear stage as one PtMatVecMult with
    the ModDown hoisted (Sec. 5.2) and the EvalMod products as NewMult
    (Sec. 5.1): eager and two graph replays equal the oracle's run of the
    same plan."""
    from paper_2112_06396_amd import trace
    pr, ctx = _get((12, 10, 4, 3), 4)
    plan = trace.bootstrap_plan(pr.L, counts=(2, 2, 3), strides=(1, 4, 16), evalmod_levels=3, hoisted=True,
                                new_mult=True)
    g = synth.rng(210)
    x0 = _rand_ct(pr, pr.L, 211)
    diag = {d: synth.uniform_residues(g, pr.key_mods(), pr.n) for d in plan.diagonals}
    keys = {k: _rand_ksk(pr, 330 + i) for i, k in enumerate(plan.rotations)}
    rlk = _rand_ksk(pr, 329)
    ref = _oracle_plan(pr, plan, x0, diag, keys, rlk)
    bufs = trace.TraceBuffers(plan, pr.n)
    bufs.view("x0", pr.L).copy_(dev(x0))
    ddiag = {d: dev(v) for d, v in diag.items()}
    dext = trace.ext_diagonals(plan, ddiag, pr.L)
    dkeys = {k: dev(v) for k, v in keys.items()}
    drlk = dev(rlk)
    out = trace.run_plan(ctx, plan, bufs, ddiag, dkeys, drlk, diag_ext=dext)
    assert np.array_equal(host(out), ref)
    gr = trace.capture(ctx, plan, bufs, ddiag, dkeys, drlk, diag_ext=dext)
    for rep in range(2):
        for name, t in bufs.ct.items():
            if name != "x0":
                t.zero_()
        torch.cuda.synchronize()
        gr.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(bufs.view(plan.out, plan.out_level)), ref), rep


def test_full_trace_graph_equals_eager():
    """The bootstrapping-shaped trace at N=2^16, L=35 -> 9, K=12, dnum=3
    (120 key-switches, 80 rotation keys + one relinearization key): the
    captured hipGraph's output equals the eager run's, twice in a row."""
    from paper_2112_06396_amd import trace
    hks = H()
    pq = hks.hks_gen_primes(50, 17, 47)
    ctx = hks.Context(16, pq[:35], pq[35:], 3, max_batch=16)
    try:
        plan = trace.bootstrap_plan(35)
        n = ctx.n
        keymods = pq
        bufs = trace.TraceBuffers(plan, n)
        bufs.view("x0", 35).copy_(synth.device_residues(pq[:35], (2,), n, 1))
        diag = {d: synth.device_residues(pq[:35], (), n, 10 + i) for i, d in enumerate(plan.diagonals)}
        keys = {k: synth.device_residues(keymods, (3, 2), n, 1000 + i) for i, k in enumerate(plan.rotations)}
        rlk = synth.device_residues(keymods, (3, 2), n, 999)
        eager = trace.run_plan(ctx, plan, bufs, diag, keys, rlk).clone()
        gr = trace.capture(ctx, plan, bufs, diag, keys, rlk)
        for rep in range(2):
            bufs.view(plan.out, plan.out_level).zero_()
            torch.cuda.synchronize()
            gr.replay()
            torch.cuda.synchronize()
            assert torch.equal(bufs.view(plan.out, plan.out_level).view(torch.int64), eager.view(torch.int64)), rep
        del gr
    finally:
        torch.cuda.synchronize()
        ctx.close()


# ------------------------------------------------------------------ serving loop


@pytest.mark.parametrize("seeded", [False, True])
def test_serving_results_same_alone_and_in_the_mix(seeded):
    """Requests of two ring degrees and mixed levels and ops, served with
    continuous batching on two lanes under a key budget that forces
    evictions, give exactly the bits of the same requests served one at a
    time; a sample of them also equals the oracle (Algorithms 2 and 3).
    With seeded keys the store holds and uploads only the rows b_j."""
    import copy
    from paper_2112_06396_amd import serving
    hks = H()
    prs = {12: O.make_params(12, 8, 3, 3), 13: O.make_params(13, 8, 3, 3)}
    n_clients = 6
    reqs = serving.poisson_requests(48, rate=2e5, n_clients=n_clients, log_ns=(12, 13), levels=(3, 8), seed=5)
    host_np, host_keys, seeds = {}, {}, ({} if seeded else None)
    for c in range(n_clients):
        ln = 12 if c % 2 == 0 else 13
        for j, kind in enumerate(("rot", "rlk")):
            k = _rand_ksk(prs[ln], 400 + 2 * c + j)
            if seeded:
                sd = 0x5E000 + 2 * c + j
                seeds[(c, kind, ln)] = sd
                k = np.stack([O.expand_key_a(prs[ln], sd), k[:, 1]], axis=1)
                store = np.ascontiguousarray(k[:, 1])
            else:
                store = k
            host_np[(c, kind, ln)] = k
            host_keys[(c, kind, ln)] = torch.from_numpy(store.view(np.int64)).view(torch.uint64).pin_memory()
    inputs_np, inputs = {}, {}
    for ln, pr in prs.items():
        for level in range(3, 9):
            cts = [_rand_ct(pr, level, 500 + 10 * level + i + ln) for i in range(2)]
            inputs_np[(ln, level)] = cts
            inputs[(ln, level)] = [dev(c) for c in cts]
    params = {ln: (pr.q, pr.p, 3) for ln, pr in prs.items()}
    ks = serving.KeyStore(host_keys, budget=9 * max(t.numel() for t in host_keys.values()) * 8)
    ex = serving.HksExecutor(params, lanes=2, max_batch=4, slots_per_n=len(reqs), keystore=ks, inputs=inputs,
                             seeds=seeds)
    try:
        eng = serving.Engine(ex, lanes=2, max_batch=4)
        alone_reqs = copy.deepcopy(reqs)
        eng.run(reqs)
        torch.cuda.synchronize()
        mix = {r.rid: host(ex.out_view(r)) for r in reqs}
        assert ks.uploads > len(host_keys)  # some keys were evicted and uploaded again
        eng.run(alone_reqs, one_at_a_time=True)
        torch.cuda.synchronize()
        for r in alone_reqs:
            assert np.array_equal(host(ex.out_view(r)), mix[r.rid]), r
        for r in reqs[:6]:
            pr = prs[r.log_n]
            pool = inputs_np[(r.log_n, r.level)]
            a = pool[r.rid % len(pool)]
            if r.op == "rotate":
                ref = O.rotate(pr, a, r.level, pow(5, -r.k, 2 * pr.n), host_np[(r.client, "rot", r.log_n)])
            else:
                b = pool[(r.rid + 1) % len(pool)]
                ref = O.mult_relin(pr, a, b, r.level, host_np[(r.client, "rlk", r.log_n)], True)
            assert np.array_equal(mix[r.rid], ref), r
    finally:
        ex.close()


@pytest.mark.parametrize("name,max_batch,n", [("cfg1", 4, 6), ("n13", 3, 4)])
def test_batch_mult_relin_seeded_equals_oracle(name, max_batch, n):
    """Mult + relinearization + Rescale with seeded keys (rows b_j only)
    equals the oracle's with the full keys (expanded rows a_j, rows b_j), in
    batched steps of max_batch."""
    pr, ctx = _get(name, max_batch)
    hks = H()
    level = pr.L
    seeds = [0x7E00 + i for i in range(n)]
    b_rows = [_rand_ksk(pr, 730 + i)[:, 1].copy() for i in range(n)]
    c1 = [_rand_ct(pr, level, 740 + i) for i in range(n)]
    c2 = [_rand_ct(pr, level, 750 + i) for i in range(n)]
    outs = [hks.empty((2, level - 1, pr.n)) for _ in range(n)]
    hks.hks_batch_mult_relin_seeded(ctx, [dev(c) for c in c1], [dev(c) for c in c2], level, seeds,
                                    [dev(b) for b in b_rows], True, outs)
    for i in range(n):
        full = np.stack([O.expand_key_a(pr, seeds[i]), b_rows[i]], axis=1)
        assert np.array_equal(host(outs[i]), O.mult_relin(pr, c1[i], c2[i], level, full, True)), i


@pytest.mark.parametrize("name,max_batch,n", [("cfg1", 4, 6), ("n13", 3, 4)])
def test_batch_mult_relin_equals_oracle(name, max_batch, n):
    pr, ctx = _get(name, max_batch)
    hks = H()
    for rs, level in ((True, pr.L), (False, pr.L - 1)):
        c1 = [_rand_ct(pr, level, 600 + i) for i in range(n)]
        c2 = [_rand_ct(pr, level, 620 + i) for i in range(n)]
        rlks = [_rand_ksk(pr, 640 + (i % 2)) for i in range(n)]
        drl = [dev(k) for k in rlks]
        outs = [hks.empty((2, level - (1 if rs else 0), pr.n)) for _ in range(n)]
        hks.hks_batch_mult_relin(ctx, [dev(c) for c in c1], [dev(c) for c in c2], level, drl, rs, outs)
        for i in range(n):
            assert np.array_equal(host(outs[i]), O.mult_relin(pr, c1[i], c2[i], level, rlks[i], rs)), (rs, i)


# ------------------------------------------------------------------ seeded keys


@pytest.mark.parametrize("name", ["n10", "cfg1", "cfg2"])
def test_expand_key_a_equals_oracle(name):
    pr, ctx = _get(name)
    hks = H()
    for seed in (0, 0xC0FFEE, (1 << 64) - 1):
        a = hks.empty((pr.dnum, pr.L + pr.K, pr.n))
        hks.hks_expand_key_a(ctx, seed, a)
        assert np.array_equal(host(a), O.expand_key_a(pr, seed)), seed


@pytest.mark.parametrize("name", ["n10", "cfg1", "n13", "cfg2"])
def test_rotate_seeded_equals_oracle(name):
    """Rotate with a seeded key (rows a_j regenerated in the key-switch
    kernel) equals the oracle's Rotate with the full key."""
    pr, ctx = _get(name)
    hks = H()
    seed = 0x5EED_0000 + pr.log_n
    b_rows = _rand_ksk(pr, 700)[:, 1].copy()
    full = np.stack([O.expand_key_a(pr, seed), b_rows], axis=1)
    for level in sorted({pr.L, pr.alpha + 1, 1}):
        ct = _rand_ct(pr, level, 701 + level)
        g = hks.hks_galois_for_rotation(3, pr.log_n)
        out = hks.empty((2, level, pr.n))
        hks.hks_rotate_seeded(ctx, dev(ct), level, g, seed, dev(b_rows), out)
        assert np.array_equal(host(out), O.rotate(pr, ct, level, g, full)), level


@pytest.mark.parametrize("name,max_batch", [("cfg1", 4), ("cfg2", 8)])
def test_batch_rotate_seeded_equals_oracle(name, max_batch):
    pr, ctx = _get(name, max_batch)
    hks = H()
    n_ct, level = 5, pr.L
    seeds = [0xABC0 + i for i in range(n_ct)]
    b_rows = [_rand_ksk(pr, 710 + i)[:, 1].copy() for i in range(n_ct)]
    cts = [_rand_ct(pr, level, 720 + i) for i in range(n_ct)]
    gals = [hks.hks_galois_for_rotation(1 + i, pr.log_n) for i in range(n_ct)]
    outs = [hks.empty((2, level, pr.n)) for _ in range(n_ct)]
    hks.hks_batch_rotate_seeded(ctx, [dev(c) for c in cts], level, gals, seeds, [dev(b) for b in b_rows], outs)
    for i in range(n_ct):
        full = np.stack([O.expand_key_a(pr, seeds[i]), b_rows[i]], axis=1)
        assert np.array_equal(host(outs[i]), O.rotate(pr, cts[i], level, gals[i], full)), i


# ------------------------------------------------------------------ PtMatVecMult with one ModDown


@pytest.mark.parametrize("name,ks", [("n10", (1, 2, -5)), ("cfg1", (1, 3)), ("n13", (2, 7, 9, -3, 11)),
                                     ("cfg2", tuple(range(1, 13)))])
def test_ptmatvec_equals_oracle(name, ks):
    """sum_i M_i * Rotate_i(ct) with the ModDown hoisted (one fused launch over
    all rotations, one ModDown) equals the oracle's algorithm bit for bit,
    at the top level and one with a short last digit."""
    pr, ctx = _get(name)
    hks = H()
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in ks]
    ksks = [_rand_ksk(pr, 800 + i) for i in range(len(ks))]
    dk = [dev(k) for k in ksks]
    for level in sorted({pr.L, pr.alpha + 1}):
        g = synth.rng(810 + level)
        ct = _rand_ct(pr, level, 811 + level)
        pts = [synth.uniform_residues(g, pr.ext_mods(level), pr.n) for _ in ks]
        out = hks.empty((2, level, pr.n))
        hks.hks_ptmatvec(ctx, dev(ct), level, gals, dk, [dev(p) for p in pts], out)
        assert np.array_equal(host(out), O.ptmatvec(pr, ct, level, gals, ksks, pts)), level


# ------------------------------------------------------------------ NewMult (key-switch ModDown merged with Rescale)


@pytest.mark.parametrize("name", ["n10", "n11", "cfg1", "n13", "cfg2", (16, 35, 12, 3)])
def test_new_mult_equals_oracle(name):
    """NewMult (ModDown by P q_(level-1) inside the key-switch) equals the
    oracle's, at the top level, at a level whose last digit is short and at
    level 2 (one output limb); a plain Mult on the same context afterwards
    is unaffected by the workspace the NewMult used."""
    pr, ctx = _get(name)
    hks = H()
    rlk = _rand_ksk(pr, 900)
    drlk = dev(rlk)
    for level in sorted({pr.L, pr.alpha + 1, 2}, reverse=True):
        c1, c2 = _rand_ct(pr, level, 901 + level), _rand_ct(pr, level, 951 + level)
        out = hks.empty((2, level - 1, pr.n))
        hks.hks_new_mult(ctx, dev(c1), dev(c2), level, drlk, out)
        assert np.array_equal(host(out), O.new_mult(pr, c1, c2, level, rlk)), level
    level = pr.L
    c1, c2 = _rand_ct(pr, level, 990), _rand_ct(pr, level, 991)
    o = hks.empty((2, level - 1, pr.n))
    hks.hks_mult_relin(ctx, dev(c1), dev(c2), level, drlk, True, o)
    assert np.array_equal(host(o), O.mult_relin(pr, c1, c2, level, rlk, True))


def test_new_mult_rejects_level_one_and_aliasing():
    pr, ctx = _get("n10")
    hks = H()
    c1, c2 = dev(_rand_ct(pr, 2, 1)), dev(_rand_ct(pr, 2, 2))
    rlk = dev(_rand_ksk(pr, 3))
    for args in ((c1, c2, 1, rlk, hks.empty((2, 1, pr.n))), (c1, c2, 2, rlk, c1), (c1, c2, 2, rlk, c2)):
        with pytest.raises(hks.HksError) as e:
            hks.hks_new_mult(ctx, *args)
        assert e.value.status == hks.HKS_EINVAL


# ------------------------------------------------------------------ input checks and C-ABI graphs


def test_canonical_checks_reject_out_of_range_inputs():
    """With checks on, a ciphertext word equal to its modulus, or a key word
    above it, makes the call return HKS_ERANGE before any work; canonical
    inputs give the same bits as with checks off; checks off accept (and do
    not look at) the bad input."""
    pr, ctx = _get("n10")
    hks = H()
    level = pr.L
    ct = _rand_ct(pr, level, 1200)
    ksk = _rand_ksk(pr, 1201)
    g = hks.hks_galois_for_rotation(1, pr.log_n)
    out = hks.empty((2, level, pr.n))
    try:
        hks.hks_set_check(ctx, True)
        hks.hks_rotate(ctx, dev(ct), level, g, dev(ksk), out)
        assert np.array_equal(host(out), O.rotate(pr, ct, level, g, ksk))
        bad = ct.copy()
        bad[1, level - 1, 77] = pr.q[level - 1]
        with pytest.raises(hks.HksError) as e:
            hks.hks_rotate(ctx, dev(bad), level, g, dev(ksk), out)
        assert e.value.status == hks.HKS_ERANGE
        badk = ksk.copy()
        badk[pr.dnum - 1, 0, pr.L + pr.K - 1, 5] = np.uint64((1 << 63) + 3)
        with pytest.raises(hks.HksError) as e:
            hks.hks_rotate(ctx, dev(ct), level, g, dev(badk), out)
        assert e.value.status == hks.HKS_ERANGE
        x = synth.uniform_residues(synth.rng(1202), pr.q[:2], pr.n)
        x[1, 3] = pr.q[1] + 1
        with pytest.raises(hks.HksError) as e:
            hks.hks_ntt(ctx, dev(x), 0, 2)
        assert e.value.status == hks.HKS_ERANGE
        # a seeded relinearization key's rows b_j, one word above its modulus
        brow = ksk[:, 1].copy()
        brow[0, pr.L, 9] = pr.p[0]
        mo = hks.empty((2, level - 1, pr.n))
        with pytest.raises(hks.HksError) as e:
            hks.hks_batch_mult_relin_seeded(ctx, [dev(ct)], [dev(ct)], level, [7], [dev(brow)], True, [mo])
        assert e.value.status == hks.HKS_ERANGE
    finally:
        hks.hks_set_check(ctx, False)
    hks.hks_rotate(ctx, dev(bad), level, g, dev(ksk), out)  # unchecked: runs
    torch.cuda.synchronize()


def test_modmul_rate_is_measured():
    """The measurement aid returns a plausible products-per-second figure
    (between 0.1 and 20 T/s on one device) and rejects zero rounds."""
    pr, ctx = _get("cfg1")
    hks = H()
    r = hks.hks_modmul_rate(ctx, 64)
    assert 1e11 < r < 2e13, r
    with pytest.raises(hks.HksError) as e:
        hks.hks_modmul_rate(ctx, 0)
    assert e.value.status == hks.HKS_EINVAL


def test_c_abi_graph_replays_equal_eager():
    """hks_graph_begin/end/launch: a Rotate and a hoisted rotation recorded
    on a stream and replayed three times, with eager calls and buffer
    clearing in between, give the eager results every time; checks on
    refuse a capturing stream."""
    pr, ctx = _get("cfg1", 4)
    hks = H()
    level = pr.L
    ct = dev(_rand_ct(pr, level, 1300))
    keys = [dev(_rand_ksk(pr, 1301 + i)) for i in range(3)]
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in (1, 2, -3)]
    o1 = hks.empty((2, level, pr.n))
    oh = [hks.empty((2, level, pr.n)) for _ in range(3)]
    hks.hks_rotate(ctx, ct, level, gals[0], keys[0], o1)
    hks.hks_hrotate(ctx, ct, level, gals, keys, oh)
    ref1, refh = host(o1).copy(), [host(t).copy() for t in oh]
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    hks.hks_graph_begin(s)
    try:
        hks.hks_set_check(ctx, True)
        with pytest.raises(hks.HksError) as e:
            hks.hks_rotate(ctx, ct, level, gals[0], keys[0], o1, s)
        assert e.value.status == hks.HKS_EUNSUPPORTED
    finally:
        hks.hks_set_check(ctx, False)
    hks.hks_rotate(ctx, ct, level, gals[0], keys[0], o1, s)
    hks.hks_hrotate(ctx, ct, level, gals, keys, oh, s)
    graph = hks.hks_graph_end(s)
    other = hks.empty((2, level, pr.n))
    for rep in range(3):
        for t in [o1] + oh:
            t.zero_()
        hks.hks_rotate(ctx, ct, level, gals[1], keys[1], other)
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        assert np.array_equal(host(o1), ref1), rep
        for i in range(3):
            assert np.array_equal(host(oh[i]), refh[i]), (rep, i)
    graph.close()
