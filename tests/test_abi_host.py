"""Host-side checks of the C ABI (no GPU): the library loads, exports every
symbol include/hks.h declares, and its host helpers and argument validation
behave as documented.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hks():
    from paper_2112_06396_amd import hks as H
    if not os.path.exists(H.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return H


def _declared(header="hks.h", prefix="hks_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(hks):
    lib = hks.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(hks.EXPORTS) == declared
    declared32 = _declared("hks32.h", "hks32_")
    assert len(declared32) == 6
    for name in declared32:
        assert hasattr(lib, name), name
    assert sorted(hks.EXPORTS32) == declared32


def test_gen_primes_matches_oracle_rule(hks):
    for bits, log_step, cnt in ((50, 17, 48), (50, 13, 10)):
        assert hks.hks_gen_primes(bits, log_step, cnt) == [int(v) for v in O.gen_primes(bits, log_step, cnt)]
    with pytest.raises(hks.HksError):
        hks.hks_gen_primes(50, 60, 3)


def test_galois_helpers(hks):
    for log_n in (10, 12, 16):
        two_n = 2 << log_n
        assert hks.hks_galois_for_rotation(1, log_n) == pow(5, -1, two_n)
        assert hks.hks_galois_for_rotation(-1, log_n) == 5
        assert hks.hks_galois_for_rotation(3, log_n) == pow(5, -3, two_n)
        assert hks.hks_galois_for_rotation(0, log_n) == 1
        assert hks.hks_galois_conjugate(log_n) == two_n - 1


def test_strerror(hks):
    assert hks.strerror(0) == "ok"
    assert hks.strerror(-1) == "invalid argument"
    assert "unknown" in hks.strerror(-99)


def _create(hks, log_n, q, p, dnum, max_batch=0):
    qa = (ctypes.c_uint64 * len(q))(*q)
    pa = (ctypes.c_uint64 * len(p))(*p)
    prm = hks._Params(log_n, len(q), len(p), dnum, qa, pa, max_batch)
    h = ctypes.c_void_p()
    return hks.lib().hks_create(ctypes.byref(prm), 0, ctypes.byref(h))


def test_create_rejects_invalid_parameters(hks):
    primes = hks.hks_gen_primes(50, 17, 12)
    q, p = primes[:6], primes[6:9]
    EINVAL = hks.HKS_EINVAL
    assert _create(hks, 9, q, p, 3) == EINVAL             # log_n out of range
    assert _create(hks, 17, q, p, 3) == EINVAL
    assert _create(hks, 12, q, p[:1], 3) == EINVAL        # K < alpha = 2
    assert _create(hks, 12, q, p, 0) == EINVAL            # dnum = 0
    assert _create(hks, 12, q, p, 7) == EINVAL            # dnum > L
    assert _create(hks, 12, q[:5] + [q[0]], p, 3) == EINVAL  # repeated prime
    assert _create(hks, 12, q[:5] + [q[5] + 2], p, 3) == EINVAL  # not prime / not 1 mod 2N
    small = [int(v) for v in O.gen_primes(40, 17, 1)]
    assert _create(hks, 12, q[:5] + small, p, 3) == EINVAL  # below 2^49
    assert _create(hks, 12, q, p, 3, max_batch=17) == EINVAL  # more batch slots than a launch holds
    rc = hks.lib().hks_create(None, 0, ctypes.byref(ctypes.c_void_p()))
    assert rc == EINVAL


def test_calls_reject_null_context(hks):
    lib = hks.lib()
    assert lib.hks_ntt(None, None, 0, 1, None) == hks.HKS_EINVAL
    assert lib.hks_rotate(None, None, 1, 5, None, None, None) == hks.HKS_EINVAL
    out = ctypes.c_uint64()
    assert lib.hks_query(None, hks.HKS_Q_N, 0, ctypes.byref(out)) == hks.HKS_EINVAL
    lib.hks_destroy(None)


def _create32(hks, log_n, q, p, dnum):
    qa = (ctypes.c_uint32 * len(q))(*q)
    pa = (ctypes.c_uint32 * len(p))(*p)
    prm = hks._Params32(log_n, len(q), len(p), dnum, qa, pa)
    h = ctypes.c_void_p()
    return hks.lib().hks32_create(ctypes.byref(prm), 0, ctypes.byref(h))


def test_create32_rejects_invalid_parameters(hks):
    """The 32-bit-word context: primes must lie in (2^20, 2^30), be 1 mod 2N,
    prime and distinct; K >= alpha; dnum in [1, L]."""
    primes = hks.hks_gen_primes(30, 17, 12)
    assert all(v < (1 << 30) for v in primes)
    q, p = primes[:6], primes[6:9]
    EINVAL = hks.HKS_EINVAL
    assert _create32(hks, 9, q, p, 3) == EINVAL
    assert _create32(hks, 12, q, p[:1], 3) == EINVAL              # K < alpha
    assert _create32(hks, 12, q, p, 0) == EINVAL
    assert _create32(hks, 12, q[:5] + [q[0]], p, 3) == EINVAL     # repeated
    assert _create32(hks, 12, q[:5] + [q[5] + 2], p, 3) == EINVAL
    big = hks.hks_gen_primes(31, 17, 1)                           # 2^30 < q < 2^31: 4q overflows a word
    assert _create32(hks, 12, q[:5] + [v & 0xFFFFFFFF for v in big], p, 3) == EINVAL
    lib = hks.lib()
    assert lib.hks32_create(None, 0, ctypes.byref(ctypes.c_void_p())) == EINVAL
    assert lib.hks32_rotate(None, None, 1, 5, None, None, None) == EINVAL
    assert lib.hks32_ntt(None, None, 0, 1, None) == EINVAL
    lib.hks32_destroy(None)


def test_binding_rejects_undersized_tensors(hks, monkeypatch):
    """The binding checks every tensor against the words the C call touches
    (computed from N, L, K, dnum and the level) before a pointer is formed,
    so a short tensor never reaches a kernel.  Runs on the CPU with the
    library replaced by a stub that records the calls (the tensors' device
    check is lifted for the test, and no pointer reaches C code)."""
    import types

    import torch
    calls = []

    class StubLib:
        def __getattr__(self, name):
            def f(*args):
                calls.append(name)
                return hks.HKS_OK
            return f

    monkeypatch.setattr(hks, "lib", lambda: StubLib())
    monkeypatch.setattr(hks, "_on_device", lambda t: True)
    monkeypatch.setattr(hks, "_stream", lambda s: ctypes.c_void_p(0))
    ctx = types.SimpleNamespace(n=1024, L=6, K=2, dnum=3, handle=None)
    n, L, K, dnum = ctx.n, ctx.L, ctx.K, ctx.dnum
    M = L + K

    def t(words):
        return torch.zeros(words, dtype=torch.int64)

    def short(fn):
        with pytest.raises(hks.HksSizeError):
            fn()

    def sized(fn):  # right size: the call goes through
        n_calls = len(calls)
        fn()
        assert len(calls) == n_calls + 1

    key, keyb = dnum * 2 * M * n, dnum * M * n
    for level in (6, 5, 3, 1):
        ct = 2 * level * n
        beta = -(-level // 2)
        for good, call in (
            (True, lambda k, c, o: hks.hks_rotate(ctx, t(c), level, 5, t(k), t(o))),
            (True, lambda k, c, o: hks.hks_rotate_seeded(ctx, t(c), level, 5, 1, t(k // 2), t(o))),
            (True, lambda k, c, o: hks.hks_batch_rotate(ctx, [t(c)], level, [5], [t(k)], [t(o)])),
            (True, lambda k, c, o: hks.hks_hrotate(ctx, t(c), level, [5, 25], [t(key), t(k)], [t(ct), t(o)])),
            (True, lambda k, c, o: hks.hks_keyswitch(ctx, t(c // 2), level, t(k), t(o))),
            (True, lambda k, c, o: hks.hks_mult_relin(ctx, t(c), t(ct), level, t(k), False, t(o))),
        ):
            sized(lambda: call(key, ct, ct))
            short(lambda: call(key - 1, ct, ct))
            short(lambda: call(key, ct - 1, ct))
            short(lambda: call(key, ct, ct - 1))
        # key built for another K or dnum
        short(lambda: hks.hks_rotate(ctx, t(ct), level, 5, t(2 * 2 * M * n), t(ct)))
        short(lambda: hks.hks_rotate(ctx, t(ct), level, 5, t(dnum * 2 * (L + 1) * n), t(ct)))
        # the extended digits and the P limbs
        sized(lambda: hks.hks_modup(ctx, t(level * n), level, t(beta * (level + K) * n)))
        short(lambda: hks.hks_modup(ctx, t(level * n), level, t(beta * (level + K) * n - 1)))
        sized(lambda: hks.hks_moddown(ctx, t((level + K) * n), level, t(level * n)))
        short(lambda: hks.hks_moddown(ctx, t(level * n), level, t(level * n)))
        sized(lambda: hks.hks_ksk_inner(ctx, t(beta * (level + K) * n), level, t(key), t(2 * (level + K) * n)))
        short(lambda: hks.hks_ksk_inner(ctx, t(beta * (level + K) * n), level, t(key), t(2 * level * n)))
        sized(lambda: hks.hks_ptmatvec(ctx, t(ct), level, [5], [t(key)], [t((level + K) * n)], t(ct)))
        short(lambda: hks.hks_ptmatvec(ctx, t(ct), level, [5], [t(key)], [t(level * n)], t(ct)))
        if level >= 2:
            # outputs one limb shorter after a Rescale, and no shorter
            sized(lambda: hks.hks_rescale(ctx, t(ct), level, t(2 * (level - 1) * n)))
            short(lambda: hks.hks_rescale(ctx, t(ct), level, t(2 * (level - 1) * n - 1)))
            sized(lambda: hks.hks_new_mult(ctx, t(ct), t(ct), level, t(key), t(2 * (level - 1) * n)))
            short(lambda: hks.hks_new_mult(ctx, t(ct), t(ct), level, t(key), t(2 * (level - 1) * n - 1)))
            short(lambda: hks.hks_ptmult(ctx, t(ct), t(level * n), level, False, t(2 * (level - 1) * n)))
            sized(lambda: hks.hks_ptmult(ctx, t(ct), t(level * n), level, True, t(2 * (level - 1) * n)))
            short(lambda: hks.hks_batch_mult_relin(ctx, [t(ct)], [t(ct)], level, [t(key)], True,
                                                   [t(2 * (level - 1) * n - 1)]))
            short(lambda: hks.hks_batch_mult_relin_seeded(ctx, [t(ct)], [t(ct)], level, [3], [t(keyb - 1)], True,
                                                          [t(2 * (level - 1) * n)]))
    short(lambda: hks.hks_ntt(ctx, t(3 * n - 1), 2, 3))
    sized(lambda: hks.hks_ntt(ctx, t(3 * n), 2, 3))
    short(lambda: hks.hks_intt(ctx, t(n), 0, 2))
    short(lambda: hks.hks_automorph(ctx, t(2 * n), t(2 * n - 1), 0, 2, 5))
    short(lambda: hks.hks_expand_key_a(ctx, 1, t(keyb - 1)))
    sized(lambda: hks.hks_expand_key_a(ctx, 1, t(keyb)))
    short(lambda: hks.hks_add(ctx, t(3 * 4 * n), t(3 * 4 * n), 4, 3, t(2 * 4 * n)))
    # the 32-bit path
    t32 = lambda words: torch.zeros(words, dtype=torch.int32)  # noqa: E731
    with pytest.raises(hks.HksSizeError):
        hks.hks32_rotate(ctx, t32(2 * 6 * n), 6, 5, t32(key - 1), t32(2 * 6 * n))
    with pytest.raises(hks.HksSizeError):
        hks.hks32_hrotate(ctx, t32(2 * 6 * n), 6, [5], [t32(key)], [t32(2 * 5 * n)])
    with pytest.raises(hks.HksSizeError):
        hks.hks32_ntt(ctx, t32(n - 1), 0, 1)
