"""Bootstrapping's linear layers with the real factored DFT (Sec. 3) on the
GPU: the device encoder against the oracle's, the PtMatVecMult diagonal
without rotation, CoeffToSlot / SlotToCoeff step by step against the oracle
(bit for bit, with the oracle's keys and encoded diagonals) and through
decryption, and a bootstrapping-shaped plan with the DFT's rotation offsets.
"""
import numpy as np
import pytest
import torch

from oracle import encoding as C
from oracle import oracle as O
from paper_2112_06396_amd import synth

pytestmark = pytest.mark.gpu

_CTX = {}


def _get(cfg, max_batch=1):
    from paper_2112_06396_amd import hks
    key = (cfg, max_batch)
    if key not in _CTX:
        log_n, L, K, dnum = cfg
        pr = O.make_params(log_n, L, K, dnum)
        _CTX[key] = (pr, hks.Context(log_n, pr.q, pr.p, dnum, max_batch=max_batch))
    return _CTX[key]


@pytest.fixture(scope="module", autouse=True)
def _cleanup():
    yield
    torch.cuda.synchronize()
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


def _z(g, n):
    return g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)


def _dev_slots(z):
    return torch.from_numpy(np.ascontiguousarray(z, dtype=np.complex128)).cuda()


def _int_coeffs(pr, pt, mods):
    """Integer coefficients of an evaluation-form plaintext (every limb must
    agree on a small centered value)."""
    c = O.centered_small(O.intt(pt, pr.log_n, mods), mods, 1 << 62)
    assert c is not None, "limbs disagree: not the residues of one integer polynomial"
    return c


@pytest.mark.parametrize("cfg", [(10, 6, 2, 3), (12, 4, 2, 2), (16, 24, 8, 3)])
def test_encode_equals_oracle(cfg):
    """hks_encode over Q_L U P and over the first limbs: exact on slots that
    decode from an integer polynomial (scale 1); on random slots at scale
    2^40 every coefficient within one unit of the oracle's (two fp64
    evaluation orders can round a near-tie differently) and almost all equal."""
    pr, ctx = _get(cfg)
    hks = H()
    n = pr.n // 2
    g = synth.rng(500 + pr.log_n)
    m = synth.small_uniform(g, pr.n, 1 << 20)
    out = hks.empty((pr.L + pr.K, pr.n))
    hks.hks_encode(ctx, _dev_slots(C.decode(m, 1.0)), 1.0, pr.L, True, out)
    assert np.array_equal(_int_coeffs(pr, host(out), pr.ext_mods(pr.L)), m)
    z = _z(g, n)
    want = C.encode(z, 2.0 ** 40)
    for level, with_p in ((pr.L, True), (max(1, pr.L // 2), False)):
        mods = pr.ext_mods(level) if with_p else pr.q[:level]
        out = hks.empty((len(mods), pr.n))
        hks.hks_encode(ctx, _dev_slots(z), 2.0 ** 40, level, with_p, out)
        got = _int_coeffs(pr, host(out), mods)
        diff = np.abs(got - want)
        assert diff.max() <= 1
        assert np.count_nonzero(diff) <= max(4, pr.n // 500)


def test_encode_rejects_bad_arguments():
    pr, ctx = _get((10, 6, 2, 3))
    hks = H()
    z = _dev_slots(np.zeros(pr.n // 2))
    out = hks.empty((pr.L + pr.K, pr.n))
    for scale, level in ((0.0, 1), (-1.0, 1), (float("inf"), 1), (1.0, 0), (1.0, pr.L + 1)):
        with pytest.raises(hks.HksError) as e:
            hks.hks_encode(ctx, z, scale, level, True, out)
        assert e.value.status == hks.HKS_EINVAL


def test_ptmatvec_diagonal_without_rotation():
    """Offset 0 alone equals PtMult bit for bit (PModUp, then an exact
    ModDown); mixed with rotations it equals the oracle's PtMatVecMult."""
    pr, ctx = _get((10, 6, 2, 3))
    hks = H()
    g = synth.rng(510)
    for level in (6, 3):
        ct = np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])
        pts = [synth.uniform_residues(g, pr.ext_mods(level), pr.n) for _ in range(3)]
        out = hks.empty((2, level, pr.n))
        hks.hks_ptmatvec(ctx, dev(ct), level, [1], [None], [dev(pts[0])], out)
        assert np.array_equal(host(out), O.ptmult(pr, ct, pts[0][:level], level, False))
        ksks = [None] + [np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                                   for _ in range(pr.dnum)]) for _ in range(2)]
        gals = [1, hks.hks_galois_for_rotation(1, pr.log_n), hks.hks_galois_for_rotation(-2, pr.log_n)]
        order = [1, 0, 2]  # the keyless term in the middle of the list
        hks.hks_ptmatvec(ctx, dev(ct), level, [gals[i] for i in order],
                         [None if ksks[i] is None else dev(ksks[i]) for i in order],
                         [dev(pts[i]) for i in order], out)
        assert np.array_equal(host(out), O.ptmatvec(pr, ct, level, [gals[i] for i in order],
                                                    [ksks[i] for i in order], [pts[i] for i in order]))
    with pytest.raises(hks.HksError):  # a keyless term must have galois 1
        hks.hks_ptmatvec(ctx, dev(ct), level, [gals[1]], [None], [dev(pts[0])], out)


def _keys(pr, s, g, factors, keys):
    for G in factors:
        for d in G:
            if d and d not in keys:
                keys[d] = O.rotation_key(pr, s, C.rotation_galois(d, pr.n), g)
    return keys


def _crt_decode(pr, s, ct, level, scale):
    from oracle import bigint as B
    mods = [int(q) for q in pr.q[:level]]
    res = O.decrypt_coef(pr, s, ct, level)
    Q = B.prod(mods)
    vals = [B.crt([int(res[i][c]) for i in range(level)], mods) for c in range(pr.n)]
    return C.decode([v - Q if v > Q // 2 else v for v in vals], scale)


def test_coeff_to_slot_and_back_on_the_gpu():
    """CoeffToSlot then SlotToCoeff at N = 2^10 (three PtMatVecMult each,
    8/15/15 then 15/15/8 diagonals including the offset-0 ones, a Rescale
    after each): every GPU step equals the oracle's bit for bit on the same
    keys and encoded diagonals; the midpoint decrypts to R w and the end to z."""
    pr, ctx = _get((10, 8, 3, 3))
    hks = H()
    g = synth.rng(520)
    s = synth.ternary(g, pr.n)
    n = pr.n // 2
    z = _z(g, n)
    scale = 2.0 ** 40
    ct = O.encrypt(pr, s, C.encode(z, scale), pr.L, g)
    keys = {}
    fwd, bwd = C.coeff_to_slot_factors(n, 3), C.slot_to_coeff_factors(n, 3)
    _keys(pr, s, g, fwd + bwd, keys)
    dkeys = {d: dev(k) for d, k in keys.items()}
    mid, lv_mid, steps_f = C.linear_layer(pr, ct, pr.L, fwd, keys)
    end, lv_end, steps_b = C.linear_layer(pr, mid, lv_mid, bwd, keys)
    by_id = {id(k): dkeys[d] for d, k in keys.items()}
    x = dev(ct)
    for level, gals, ksks, pts, pre in steps_f + steps_b:
        dks = [None if k is None else by_id[id(k)] for k in ksks]
        acc = hks.empty((2, level, pr.n))
        hks.hks_ptmatvec(ctx, x, level, gals, dks, [dev(p) for p in pts], acc)
        assert np.array_equal(host(acc), pre), level
        x = hks.empty((2, level - 1, pr.n))
        hks.hks_rescale(ctx, acc, level, x)
        if level - 1 == lv_mid:
            got_mid = host(x)
            assert np.array_equal(got_mid, mid)
    got = host(x)
    assert np.array_equal(got, end)
    want_mid = C.encode_w(z)[C.bit_reverse_perm(n)]
    assert np.max(np.abs(_crt_decode(pr, s, got_mid, lv_mid, scale) - want_mid)) < 1e-6
    assert np.max(np.abs(_crt_decode(pr, s, got, lv_end, scale) - z)) < 1e-5


def test_dft_plan_eager_and_graph_match_oracle():
    """A bootstrapping-shaped plan whose linear stages carry the factored
    DFT's rotation offsets (2^11 slots, three iterations of 3, 4 and 4
    stages) with hoisted PtMatVecMult and NewMult: eager and graph replays
    equal the oracle's run of the same plan."""
    from paper_2112_06396_amd import trace
    from test_gpu_parity import _oracle_plan
    pr, ctx = _get((12, 10, 4, 3), 4)
    plan = trace.bootstrap_plan(pr.L, evalmod_levels=2, hoisted=True, new_mult=True, dft=(pr.log_n - 1, 3))
    assert 0 not in plan.rotations
    g = synth.rng(530)
    x0 = np.stack([synth.uniform_residues(g, pr.q, pr.n) for _ in range(2)])
    diag = {d: synth.uniform_residues(g, pr.key_mods(), pr.n) for d in plan.diagonals}
    keys = {k: np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                         for _ in range(pr.dnum)]) for k in plan.rotations}
    rlk = np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                    for _ in range(pr.dnum)])
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


def test_full_size_dft_trace_graph_equals_eager():
    """The bootstrapping-shaped plan with the factored DFT's offsets at
    N = 2^16, L = 35 -> 9, K = 12, dnum = 3 (2^15 slots, three iterations:
    155 rotation keys, 350 key-switches, diagonals encoded on the device):
    one captured hipGraph replayed twice equals the eager run."""
    from paper_2112_06396_amd import hks, trace
    pq = hks.hks_gen_primes(50, 17, 47)
    ctx = hks.Context(16, pq[:35], pq[35:], 3, max_batch=16)
    try:
        n = ctx.n
        plan = trace.bootstrap_plan(35, hoisted=True, new_mult=True, dft=(15, 3))
        assert plan.key_switches == 350 and len(plan.rotations) == 155
        keys = {k: synth.device_residues(pq, (3, 2), n, 3000 + i) for i, k in enumerate(plan.rotations)}
        rlk = synth.device_residues(pq, (3, 2), n, 2999)
        gz = torch.Generator(device="cuda")
        gz.manual_seed(5)
        diag = {}
        for d in plan.diagonals:
            zs = torch.rand((n // 2, 2), generator=gz, dtype=torch.float64, device="cuda") * 2 - 1
            diag[d] = hks.empty((len(pq), n))
            hks.hks_encode(ctx, zs, 2.0 ** 40, 35, True, diag[d])
        ext = trace.ext_diagonals(plan, diag, 35)
        bufs = trace.TraceBuffers(plan, n)
        bufs.view("x0", 35).copy_(synth.device_residues(pq[:35], (2,), n, 3))
        eager = trace.run_plan(ctx, plan, bufs, {}, keys, rlk, diag_ext=ext).clone()
        gr = trace.capture(ctx, plan, bufs, {}, keys, rlk, diag_ext=ext)
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
