"""Batches of ciphertexts at uneven levels in shared launches.

hks_batch_rotate_mixed and hks_batch_mult_relin_mixed serve ciphertexts of
different limb counts in one launch sequence (every launch covers the
step's largest Q_level U P; entries below it skip the limbs they do not
have).  Each result must equal the oracle's Rotate (Algorithm 3) or Mult
(Algorithm 2) at that ciphertext's own level, word for word, and the same
call of the single-level entry points.
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


def _get(shape, max_batch):
    hks = H()
    key = (shape, max_batch)
    if key not in _CTX:
        log_n, L, K, dnum = shape
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


def dev(a):
    return H().to_device(a)


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


# (log N, L, K, dnum): alpha = 3 with a short last digit at most levels
SMALL = (13, 8, 3, 3)


@pytest.mark.parametrize("seeded", [False, True])
def test_mixed_rotate_equals_oracle_per_level(seeded):
    """Levels 8, 1, 5, 3, 7, 8, 2 (digits 3, 1, 2, 1, 3, 3, 1) in steps of
    4: each ciphertext's Rotate equals the oracle's at its level."""
    hks = H()
    pr, ctx = _get(SMALL, 4)
    levels = [8, 1, 5, 3, 7, 8, 2]
    ks = [1, -2, 3, 5, -7, 11, 2]
    cts = [_ct(pr, lv, 3000 + i) for i, lv in enumerate(levels)]
    keys = [_ksk(pr, 3100 + i) for i in range(len(levels))]
    seeds = [0xABC0 + i for i in range(len(levels))] if seeded else None
    if seeded:  # the key's rows a_j come from the seed
        keys = [np.stack([O.expand_key_a(pr, sd), k[:, 1]], axis=1) for sd, k in zip(seeds, keys)]
        d_keys = [dev(np.ascontiguousarray(k[:, 1])) for k in keys]
    else:
        d_keys = [dev(k) for k in keys]
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in ks]
    outs = [hks.empty((2, lv, pr.n)) for lv in levels]
    print(f"[mixed] rotate levels={levels} seeded={seeded}", flush=True)
    hks.hks_batch_rotate_mixed(ctx, [dev(c) for c in cts], levels, gals, d_keys, outs, seeds=seeds)
    for i, lv in enumerate(levels):
        assert np.array_equal(host(outs[i]), O.rotate(pr, cts[i], lv, gals[i], keys[i])), (i, lv)


def test_mixed_mult_equals_oracle_per_level():
    hks = H()
    pr, ctx = _get(SMALL, 4)
    levels = [8, 2, 6, 4, 3]
    c1 = [_ct(pr, lv, 3200 + i) for i, lv in enumerate(levels)]
    c2 = [_ct(pr, lv, 3300 + i) for i, lv in enumerate(levels)]
    rlks = [_ksk(pr, 3400 + i) for i in range(len(levels))]
    for rescale in (True, False):
        outs = [hks.empty((2, lv - (1 if rescale else 0), pr.n)) for lv in levels]
        print(f"[mixed] mult levels={levels} rescale={rescale}", flush=True)
        hks.hks_batch_mult_relin_mixed(ctx, [dev(c) for c in c1], [dev(c) for c in c2], levels,
                                       [dev(k) for k in rlks], rescale, outs)
        for i, lv in enumerate(levels):
            want = O.mult_relin(pr, c1[i], c2[i], lv, rlks[i], rescale)
            assert np.array_equal(host(outs[i]), want), (i, lv, rescale)
    # seeded relinearization keys
    seeds = [0x77 + i for i in range(len(levels))]
    full = [np.stack([O.expand_key_a(pr, sd), k[:, 1]], axis=1) for sd, k in zip(seeds, rlks)]
    outs = [hks.empty((2, lv - 1, pr.n)) for lv in levels]
    hks.hks_batch_mult_relin_mixed(ctx, [dev(c) for c in c1], [dev(c) for c in c2], levels,
                                   [dev(np.ascontiguousarray(k[:, 1])) for k in rlks], True, outs, seeds=seeds)
    for i, lv in enumerate(levels):
        assert np.array_equal(host(outs[i]), O.mult_relin(pr, c1[i], c2[i], lv, full[i], True)), i


def test_mixed_rotate_full_size_equals_single_level_calls():
    """N = 2^16, L = 35, K = 12, dnum = 3 (the bootstrapping trace's top
    level): levels 35, 13, 24, 1, 36 > L rejected; the mixed step equals
    hks_rotate at each level, and the oracle at level 13."""
    hks = H()
    pr, ctx = _get((16, 35, 12, 3), 4)
    levels = [35, 13, 24, 1, 30]
    gals = [hks.hks_galois_for_rotation(k, pr.log_n) for k in (1, 2, -3, 4, 5)]
    d_cts = [synth.device_residues([int(q) for q in pr.q[:lv]], (2,), pr.n, 3500 + i)
             for i, lv in enumerate(levels)]
    d_keys = [synth.device_residues([int(q) for q in pr.key_mods()], (3, 2), pr.n, 3600 + i)
              for i in range(len(levels))]
    outs = [hks.empty((2, lv, pr.n)) for lv in levels]
    print(f"[mixed] full size levels={levels}", flush=True)
    hks.hks_batch_rotate_mixed(ctx, d_cts, levels, gals, d_keys, outs)
    ref = hks.empty((2, 35, pr.n))
    for i, lv in enumerate(levels):
        r = ref.view(-1)[: 2 * lv * pr.n].view(2, lv, pr.n)
        hks.hks_rotate(ctx, d_cts[i], lv, gals[i], d_keys[i], r)
        assert torch.equal(outs[i], r), (i, lv)
    i = levels.index(13)
    assert np.array_equal(host(outs[i]), O.rotate(pr, host(d_cts[i]), 13, gals[i], host(d_keys[i])))
    with pytest.raises(hks.HksError):
        hks.hks_batch_rotate_mixed(ctx, d_cts[:1], [36], gals[:1], d_keys[:1], outs[:1])
