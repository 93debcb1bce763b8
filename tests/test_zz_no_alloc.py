"""The allocation-free Rotate (hks_rotate_noalloc) against hks_rotate.

The entry point runs the same kernels as hks_rotate with the library's fixed
device scratch array as the workspace instead of the context's.  Two calls in
a row (the second with a smaller input: a lower level, then a context of a
smaller ring degree, both reusing the scratch the first call left behind)
must equal hks_rotate word for word, and hks_rotate must equal the oracle.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2112_06396_amd import synth

pytestmark = pytest.mark.gpu


def _hks():
    from paper_2112_06396_amd import hks
    return hks


def _case(pr, level, seed):
    g = synth.rng(seed)
    ct = np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])
    ksk = np.stack([np.stack([synth.uniform_residues(g, pr.key_mods(), pr.n) for _ in range(2)])
                    for _ in range(pr.dnum)])
    return ct, ksk


def _both(hks, ctx, pr, level, k, seed, oracle):
    ct, ksk = _case(pr, level, seed)
    d_ct, d_ksk = hks.to_device(ct), hks.to_device(ksk)
    gal = hks.hks_galois_for_rotation(k, pr.log_n)
    ref = hks.empty((2, level, pr.n))
    got = hks.empty((2, level, pr.n))
    got.fill_(7)  # not the answer
    print(f"[noalloc] N=2^{pr.log_n} L={pr.L} level={level} k={k}", flush=True)
    hks.hks_rotate(ctx, d_ct, level, gal, d_ksk, ref)
    hks.hks_rotate_noalloc(ctx, d_ct, level, gal, d_ksk, got)
    torch.cuda.synchronize()
    want = hks.to_host(ref)
    assert np.array_equal(hks.to_host(got), want), (pr.log_n, level)
    if oracle:
        assert np.array_equal(want, O.rotate(pr, ct, level, gal, ksk)), (pr.log_n, level)


def test_noalloc_rotate_equals_rotate_twice_in_a_row():
    hks = _hks()
    big = O.make_params(16, 24, 8, 3)
    small = O.make_params(12, 4, 2, 2)
    with hks.Context(16, big.q, big.p, 3) as cb:
        assert hks.hks_query(cb, hks.HKS_Q_NOALLOC_MAX_BYTES) == 128 << 20
        assert hks.hks_query(cb, hks.HKS_Q_NOALLOC_BYTES, 24) == (5 * 24 + 2 * 8 + 3 * 32) * (1 << 16) * 8
        assert hks.hks_query(cb, hks.HKS_Q_NOALLOC_BYTES, 11) == (5 * 11 + 2 * 8 + 2 * 32) * (1 << 16) * 8
        # the bench shape, then a smaller level on the same scratch
        _both(hks, cb, big, 24, 1, 31, oracle=False)
        _both(hks, cb, big, 11, -3, 32, oracle=True)
        # and a repeat at the top level after the smaller one
        _both(hks, cb, big, 24, 5, 33, oracle=False)
    with hks.Context(12, small.q, small.p, 2) as cs:
        # a smaller ring degree: the scratch holds the larger calls' words
        _both(hks, cs, small, 4, 1, 34, oracle=True)
        _both(hks, cs, small, 3, 2, 35, oracle=True)


def test_noalloc_rotate_rejects_what_does_not_fit():
    hks = _hks()
    pr = O.make_params(16, 35, 12, 3)
    with hks.Context(16, pr.q, pr.p, 3) as ctx:
        need = hks.hks_query(ctx, hks.HKS_Q_NOALLOC_BYTES, 35)
        assert need > hks.HKS_NOALLOC_SCRATCH_BYTES
        ct = hks.empty((2, 35, pr.n))
        ct.zero_()
        key = hks.empty((3, 2, 47, pr.n))
        key.zero_()
        out = hks.empty((2, 35, pr.n))
        with pytest.raises(hks.HksError) as ei:
            hks.hks_rotate_noalloc(ctx, ct, 35, hks.hks_galois_for_rotation(1, 16), key, out)
        assert ei.value.status == hks.HKS_ESCRATCH
        # a level that fits runs and matches hks_rotate
        _both(hks, ctx, pr, 13, 1, 36, oracle=False)
