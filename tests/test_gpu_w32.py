"""Parity of the 32-bit-word key-switch (include/hks32.h) with the oracle
run on the same 30-bit primes: NTT / iNTT, Rotate and HRotate, bit for
bit, at small sizes (several tiles, short last digit, level 1, K above
alpha) and at N = 2^16 with the log2(QP) of the 50-bit benchmark (L = 40,
K = 14, dnum = 3)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2112_06396_amd import synth

pytestmark = pytest.mark.gpu

CFGS = {
    # name: (log_n, L, K, dnum)
    "n10": (10, 8, 3, 3),
    "n11": (11, 5, 2, 3),
    "n13": (13, 10, 4, 3),
    "n15": (15, 9, 4, 3),   # K = 4 special primes above alpha = 3
    "full": (16, 40, 14, 3),
}
_CTX = {}


def _get(name):
    from paper_2112_06396_amd import hks
    if name not in _CTX:
        log_n, L, K, dnum = CFGS[name]
        pr = O.make_params(log_n, L, K, dnum, bits=30)
        _CTX[name] = (pr, hks.Context32(log_n, pr.q, pr.p, dnum))
    return _CTX[name]


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


def host(t):
    torch.cuda.synchronize()
    return H().to_host32(t)


def _ct(pr, level, seed):
    g = synth.rng(seed)
    return np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])


def _ksk(pr, seed):
    g = synth.rng(seed)
    return np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                     for _ in range(pr.dnum)])


@pytest.mark.parametrize("name", list(CFGS))
def test_ntt_intt_equal_oracle(name):
    pr, ctx = _get(name)
    hks = H()
    mods = pr.key_mods()
    g = synth.rng(800 + pr.log_n)
    x = synth.uniform_residues(g, mods, pr.n)
    d = hks.to_device32(x)
    hks.hks32_ntt(ctx, d, 0, len(mods))
    assert np.array_equal(host(d), O.ntt(x, pr.log_n, mods))
    hks.hks32_intt(ctx, d, 0, len(mods))
    assert np.array_equal(host(d), x)
    y = synth.uniform_residues(g, mods[pr.L:], pr.n)  # the P limbs alone
    d = hks.to_device32(y)
    hks.hks32_intt(ctx, d, pr.L, pr.K)
    assert np.array_equal(host(d), O.intt(y, pr.log_n, mods[pr.L:]))


@pytest.mark.parametrize("name", list(CFGS))
def test_rotate_equals_oracle(name):
    pr, ctx = _get(name)
    hks = H()
    ksk = _ksk(pr, 810)
    dk = hks.to_device32(ksk)
    levels = sorted({pr.L, pr.alpha + 1, pr.alpha, 1} - {0})
    if name == "full":
        levels = [pr.L, 17]
    for level in levels:
        ct = _ct(pr, level, 820 + level)
        for gal in (hks.hks_galois_for_rotation(1, pr.log_n), hks.hks_galois_for_rotation(-5, pr.log_n),
                    hks.hks_galois_conjugate(pr.log_n)):
            out = hks.empty32((2, level, pr.n))
            hks.hks32_rotate(ctx, hks.to_device32(ct), level, gal, dk, out)
            assert np.array_equal(host(out), O.rotate(pr, ct, level, gal, ksk)), (level, gal)


@pytest.mark.parametrize("name", list(CFGS))
def test_hrotate_equals_oracle(name):
    """HRotate (one ModUp, r KSKInnerProds over the automorphed digits) equals
    the oracle's Algorithm 4 with the same 30-bit primes, bit for bit."""
    pr, ctx = _get(name)
    hks = H()
    # six rotations: ModDown steps of four and two
    ks = (1, -5, 3, 2, -1, 6) if name != "full" else (1, 7)
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in ks]
    ksks = [_ksk(pr, 850 + i) for i in range(len(ks))]
    dks = [hks.to_device32(k) for k in ksks]
    levels = [pr.L, 1] if name != "full" else [pr.L]
    for level in levels:
        ct = _ct(pr, level, 860 + level)
        outs = [hks.empty32((2, level, pr.n)) for _ in ks]
        hks.hks32_hrotate(ctx, hks.to_device32(ct), level, gals, dks, outs)
        want = O.hrotate(pr, ct, level, gals, ksks)
        for k, o, w in zip(ks, outs, want):
            assert np.array_equal(host(o), w), (level, k)


def test_hrotate_rejects_bad_arguments():
    pr, ctx = _get("n10")
    hks = H()
    ct = hks.to_device32(_ct(pr, 2, 870))
    k = hks.to_device32(_ksk(pr, 871))
    out = hks.empty32((2, 2, pr.n))
    for level, gals, o in ((0, [5], out), (pr.L + 1, [5], out), (2, [5, 4], out), (2, [5], ct), (2, [], out)):
        with pytest.raises(hks.HksError) as e:
            hks.hks32_hrotate(ctx, ct, level, gals, [k] * len(gals), [o] * len(gals))
        assert e.value.status == hks.HKS_EINVAL


def test_rotate_valid_key_decrypts():
    """With a real rotation key (30-bit primes) the GPU output equals the
    oracle's and decrypts to the rotated message within the noise bound."""
    pr, ctx = _get("n10")
    hks = H()
    g = synth.rng(830)
    s = synth.ternary(g, pr.n)
    gal = hks.hks_galois_for_rotation(2, pr.log_n)
    ksk = O.rotation_key(pr, s, gal, g)
    level = pr.L
    ct = O.encrypt(pr, s, synth.small_uniform(g, pr.n, 1 << 20), level, g)
    out = hks.empty32((2, level, pr.n))
    hks.hks32_rotate(ctx, hks.to_device32(ct), level, gal, hks.to_device32(ksk), out)
    got = host(out)
    assert np.array_equal(got, O.rotate(pr, ct, level, gal, ksk))
    mods = pr.q[:level]
    diff = O.sub_vec(O.decrypt_coef(pr, s, got, level),
                     O.automorph(O.decrypt_coef(pr, s, ct, level), pr.log_n, mods, gal, eval_domain=False),
                     pr.log_n, mods)
    assert O.centered_small(diff, mods, O.ks_noise_bound(pr, level, s)) is not None


def test_rotate_rejects_bad_arguments():
    pr, ctx = _get("n10")
    hks = H()
    ct = hks.to_device32(_ct(pr, 2, 840))
    k = hks.to_device32(_ksk(pr, 841))
    out = hks.empty32((2, 2, pr.n))
    for level, gal, o in ((0, 5, out), (pr.L + 1, 5, out), (2, 4, out), (2, 2 * pr.n + 1, out), (2, 5, ct)):
        with pytest.raises(hks.HksError) as e:
            hks.hks32_rotate(ctx, ct, level, gal, k, o)
        assert e.value.status == hks.HKS_EINVAL
