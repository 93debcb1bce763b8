"""Python face of the plain CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark import this module.  It wraps ``liboracle.so`` (built from
``ref.c``) with ctypes and adds the test-side pieces of CKKS that the
key-switching path itself does not contain: switching-key generation
(the Han-Ki gadget in RNS form, Eq. kskShape), encryption, decryption, and
the noise check.  Decryption convention: m' = a*s + b (Algorithms 2 and 3).

All polynomials are numpy uint64 arrays, limb-major ([limbs][N]), canonical
residues, evaluation form (bit-reversed order) unless a name says "coef".
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from paper_2112_06396_amd import synth

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)


class _CParams(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_uint32),
        ("L", ctypes.c_uint32),
        ("K", ctypes.c_uint32),
        ("dnum", ctypes.c_uint32),
        ("q", _u64p),
        ("p", _u64p),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        P = ctypes.POINTER(_CParams)
        sig = {
            "oref_is_prime": (i32, [u64]),
            "oref_gen_primes": (i32, [u32, u32, u32, _u64p]),
            "oref_psi": (u64, [u64, u32]),
            "oref_mulmod": (u64, [u64, u64, u64]),
            "oref_powmod": (u64, [u64, u64, u64]),
            "oref_ntt": (None, [_u64p, u32, _u64p, u32]),
            "oref_intt": (None, [_u64p, u32, _u64p, u32]),
            "oref_automorph": (None, [_u64p, _u64p, u32, _u64p, u32, u32, i32]),
            "oref_alpha": (u32, [P]),
            "oref_beta": (u32, [P, u32]),
            "oref_modup": (i32, [P, _u64p, u32, _u64p]),
            "oref_ksk_inner": (i32, [P, _u64p, u32, _u64p, _u64p]),
            "oref_moddown": (i32, [P, _u64p, u32, _u64p]),
            "oref_keyswitch": (i32, [P, _u64p, u32, _u64p, _u64p]),
            "oref_rotate": (i32, [P, _u64p, u32, u32, _u64p, _u64p]),
            "oref_hrotate": (i32, [P, _u64p, u32, u32, ctypes.POINTER(u32),
                                   ctypes.POINTER(_u64p), ctypes.POINTER(_u64p)]),
            "oref_rescale": (i32, [P, _u64p, u32, _u64p]),
            "oref_ptmult": (i32, [P, _u64p, _u64p, u32, i32, _u64p]),
            "oref_mult_relin": (i32, [P, _u64p, _u64p, u32, _u64p, i32, _u64p]),
            "oref_mul_vec": (None, [_u64p, _u64p, _u64p, u32, _u64p, u32]),
            "oref_add_vec": (None, [_u64p, _u64p, _u64p, u32, _u64p, u32]),
            "oref_sub_vec": (None, [_u64p, _u64p, _u64p, u32, _u64p, u32]),
            "oref_scale_vec": (None, [_u64p, _u64p, _u64p, u32, _u64p, u32]),
            "oref_lift_signed": (None, [ctypes.POINTER(ctypes.c_int64), _u64p, u32, _u64p, u32]),
            "oref_philox4x32_10": (None, [ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]),
            "oref_expand_key_a": (None, [P, u64, _u64p]),
            "oref_ptmatvec": (i32, [P, _u64p, u32, u32, ctypes.POINTER(u32), ctypes.POINTER(_u64p),
                                    ctypes.POINTER(_u64p), _u64p]),
            "oref_new_mult": (i32, [P, _u64p, _u64p, u32, _u64p, _u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_u64p)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


# ---------------------------------------------------------------------------
# Parameters (Table "CKKS FHE Parameters")
# ---------------------------------------------------------------------------

def gen_primes(bits: int, log_step: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    if lib().oref_gen_primes(bits, log_step, count, _p(out)) != 0:
        raise ValueError("prime search failed")
    return out


def is_prime(n: int) -> bool:
    return bool(lib().oref_is_prime(int(n)))


def psi(q: int, log_n: int) -> int:
    return int(lib().oref_psi(int(q), log_n))


@dataclass
class Params:
    log_n: int
    L: int
    K: int
    dnum: int
    q: np.ndarray  # [L] uint64
    p: np.ndarray  # [K] uint64

    @property
    def n(self) -> int:
        return 1 << self.log_n

    @property
    def alpha(self) -> int:
        return -(-self.L // self.dnum)

    def beta(self, level: int) -> int:
        return -(-level // self.alpha)

    def ext_mods(self, level: int) -> np.ndarray:
        return np.concatenate([self.q[:level], self.p]).astype(np.uint64)

    def key_mods(self) -> np.ndarray:
        return np.concatenate([self.q, self.p]).astype(np.uint64)

    def c(self):
        self._q = _u64(self.q)
        self._pp = _u64(self.p)
        cp = _CParams(self.log_n, self.L, self.K, self.dnum, _p(self._q), _p(self._pp))
        return ctypes.byref(cp), cp


def c_alpha(pr: Params) -> int:
    """alpha as the C oracle computes it (limbs per digit of Decomp)."""
    ref, keep = pr.c()
    a = int(lib().oref_alpha(ref))
    del keep
    return a


def c_beta(pr: Params, level: int) -> int:
    """beta at `level` limbs as the C oracle computes it (digits of Decomp)."""
    ref, keep = pr.c()
    b = int(lib().oref_beta(ref, int(level)))
    del keep
    return b


def make_params(log_n: int, L: int, K: int, dnum: int, bits: int = 50, log_step: int = 17) -> Params:
    pr = gen_primes(bits, log_step, L + K)
    return Params(log_n, L, K, dnum, pr[:L].copy(), pr[L:].copy())


# ---------------------------------------------------------------------------
# Polynomial-level operations
# ---------------------------------------------------------------------------

def ntt(x: np.ndarray, log_n: int, mods) -> np.ndarray:
    y = _u64(x).copy()
    m = _u64(mods)
    lib().oref_ntt(_p(y), log_n, _p(m), len(m))
    return y


def intt(x: np.ndarray, log_n: int, mods) -> np.ndarray:
    y = _u64(x).copy()
    m = _u64(mods)
    lib().oref_intt(_p(y), log_n, _p(m), len(m))
    return y


def automorph(x: np.ndarray, log_n: int, mods, g: int, eval_domain: bool = True) -> np.ndarray:
    x = _u64(x)
    y = np.empty_like(x)
    m = _u64(mods)
    lib().oref_automorph(_p(x), _p(y), log_n, _p(m), len(m), g, 1 if eval_domain else 0)
    return y


def _call(name, pr: Params, *args):
    ref, keep = pr.c()
    rc = getattr(lib(), name)(ref, *args)
    del keep
    if rc != 0:
        raise ValueError(f"{name} rejected its arguments")


def modup(pr: Params, a: np.ndarray, level: int) -> np.ndarray:
    a = _u64(a)
    ext = np.zeros((pr.beta(level), level + pr.K, pr.n), dtype=np.uint64)
    _call("oref_modup", pr, _p(a), level, _p(ext))
    return ext


def ksk_inner(pr: Params, ext: np.ndarray, level: int, ksk: np.ndarray) -> np.ndarray:
    ext, ksk = _u64(ext), _u64(ksk)
    uv = np.zeros((2, level + pr.K, pr.n), dtype=np.uint64)
    _call("oref_ksk_inner", pr, _p(ext), level, _p(ksk), _p(uv))
    return uv


def moddown(pr: Params, x: np.ndarray, level: int) -> np.ndarray:
    x = _u64(x)
    y = np.zeros((level, pr.n), dtype=np.uint64)
    _call("oref_moddown", pr, _p(x), level, _p(y))
    return y


def keyswitch(pr: Params, d: np.ndarray, level: int, ksk: np.ndarray) -> np.ndarray:
    d, ksk = _u64(d), _u64(ksk)
    uv = np.zeros((2, level, pr.n), dtype=np.uint64)
    _call("oref_keyswitch", pr, _p(d), level, _p(ksk), _p(uv))
    return uv


def rotate(pr: Params, ct: np.ndarray, level: int, g: int, ksk: np.ndarray) -> np.ndarray:
    ct, ksk = _u64(ct), _u64(ksk)
    out = np.zeros((2, level, pr.n), dtype=np.uint64)
    _call("oref_rotate", pr, _p(ct), level, g, _p(ksk), _p(out))
    return out


def hrotate(pr: Params, ct: np.ndarray, level: int, gs, ksks) -> list:
    ct = _u64(ct)
    ksks = [_u64(k) for k in ksks]
    outs = [np.zeros((2, level, pr.n), dtype=np.uint64) for _ in gs]
    r = len(gs)
    garr = (ctypes.c_uint32 * r)(*[int(g) for g in gs])
    karr = (_u64p * r)(*[_p(k) for k in ksks])
    oarr = (_u64p * r)(*[_p(o) for o in outs])
    _call("oref_hrotate", pr, _p(ct), level, r, garr, karr, oarr)
    return outs


def ptmatvec(pr: Params, ct: np.ndarray, level: int, gs, ksks, pts) -> np.ndarray:
    """sum_i M_i * Rotate_{g_i}(ct) with one ModDown (hoisted PtMatVecMult);
    pts[i] is M_i over Q_level U P, [level + K][N] evaluation form.  A key of
    None (with g_i = 1) is the diagonal without rotation: PModUp of ct
    itself, no key switch."""
    ct = _u64(ct)
    ksks = [None if k is None else _u64(k) for k in ksks]
    pts = [_u64(p) for p in pts]
    r = len(gs)
    out = np.zeros((2, level, pr.n), dtype=np.uint64)
    ga = (ctypes.c_uint32 * r)(*[int(g) for g in gs])
    ka = (_u64p * r)(*[_u64p() if k is None else _p(k) for k in ksks])
    pa = (_u64p * r)(*[_p(p) for p in pts])
    _call("oref_ptmatvec", pr, _p(ct), level, r, ga, ka, pa, _p(out))
    return out


def new_mult(pr: Params, ct1, ct2, level: int, rlk) -> np.ndarray:
    """Mult with the key-switch ModDown and Rescale merged into one ModDown by
    P q_(level-1) (NewMult); output [2][level - 1][N]."""
    ct1, ct2, rlk = _u64(ct1), _u64(ct2), _u64(rlk)
    out = np.zeros((2, level - 1, pr.n), dtype=np.uint64)
    _call("oref_new_mult", pr, _p(ct1), _p(ct2), level, _p(rlk), _p(out))
    return out


def rescale(pr: Params, ct: np.ndarray, level: int) -> np.ndarray:
    ct = _u64(ct)
    out = np.zeros((2, level - 1, pr.n), dtype=np.uint64)
    _call("oref_rescale", pr, _p(ct), level, _p(out))
    return out


def ptmult(pr: Params, ct: np.ndarray, pt: np.ndarray, level: int, do_rescale: bool) -> np.ndarray:
    ct, pt = _u64(ct), _u64(pt)
    out = np.zeros((2, level - (1 if do_rescale else 0), pr.n), dtype=np.uint64)
    _call("oref_ptmult", pr, _p(ct), _p(pt), level, 1 if do_rescale else 0, _p(out))
    return out


def mult_relin(pr: Params, ct1, ct2, level: int, rlk, do_rescale: bool) -> np.ndarray:
    ct1, ct2, rlk = _u64(ct1), _u64(ct2), _u64(rlk)
    out = np.zeros((2, level - (1 if do_rescale else 0), pr.n), dtype=np.uint64)
    _call("oref_mult_relin", pr, _p(ct1), _p(ct2), level, _p(rlk), 1 if do_rescale else 0, _p(out))
    return out


def mul_vec(x, y, log_n, mods):
    x, y, m = _u64(x), _u64(y), _u64(mods)
    out = np.empty_like(x)
    lib().oref_mul_vec(_p(x), _p(y), _p(out), log_n, _p(m), len(m))
    return out


def add_vec(x, y, log_n, mods):
    x, y, m = _u64(x), _u64(y), _u64(mods)
    out = np.empty_like(x)
    lib().oref_add_vec(_p(x), _p(y), _p(out), log_n, _p(m), len(m))
    return out


def sub_vec(x, y, log_n, mods):
    x, y, m = _u64(x), _u64(y), _u64(mods)
    out = np.empty_like(x)
    lib().oref_sub_vec(_p(x), _p(y), _p(out), log_n, _p(m), len(m))
    return out


def scale_vec(x, scalars, log_n, mods):
    x, s, m = _u64(x), _u64(scalars), _u64(mods)
    out = np.empty_like(x)
    lib().oref_scale_vec(_p(x), _p(s), _p(out), log_n, _p(m), len(m))
    return out


def lift_signed(v: np.ndarray, log_n: int, mods) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(v, dtype=np.int64))
    m = _u64(mods)
    out = np.zeros((len(m), 1 << log_n), dtype=np.uint64)
    lib().oref_lift_signed(v.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(out), log_n, _p(m), len(m))
    return out


# ---------------------------------------------------------------------------
# Keys, encryption, decryption (tests only)
# ---------------------------------------------------------------------------

def secret_eval(pr: Params, s: np.ndarray) -> np.ndarray:
    """ternary secret -> evaluation form over q_0..q_{L-1}, p_0..p_{K-1}."""
    mods = pr.key_mods()
    return ntt(lift_signed(s, pr.log_n, mods), pr.log_n, mods)


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter and 2-word key -> 4 words."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oref_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def expand_key_a(pr: Params, seed: int) -> np.ndarray:
    """The uniform rows a_j of a seeded switching key, [dnum][L+K][N]."""
    a = np.zeros((pr.dnum, pr.L + pr.K, pr.n), dtype=np.uint64)
    ref, keep = pr.c()
    lib().oref_expand_key_a(ref, int(seed), _p(a))
    del keep
    return a


def switch_key(pr: Params, s_hat: np.ndarray, s_from_hat: np.ndarray, g: np.random.Generator,
               uniform_a: bool = True, seed=None) -> np.ndarray:
    """Switching key from s_from to s in the Han-Ki gadget form (Eq. kskShape).

    ksk[j] = (a_j, b_j) with b_j = -a_j*s + e_j + [P]_{q_i} * s_from on the
    limbs q_i of digit j (i in [j*alpha, (j+1)*alpha)), over Q_L U P.
    Layout [dnum][2][L+K][N].  With `seed`, a_j are the seeded rows
    expand_key_a(seed)[j] (a seeded key: only the b rows need storing).
    """
    mods = pr.key_mods()
    kl = pr.L + pr.K
    ksk = np.zeros((pr.dnum, 2, kl, pr.n), dtype=np.uint64)
    P = 1
    for pk in pr.p:
        P *= int(pk)
    a_seeded = expand_key_a(pr, seed) if seed is not None else None
    for j in range(pr.dnum):
        a = a_seeded[j] if a_seeded is not None else synth.uniform_residues(g, mods, pr.n)
        e = ntt(lift_signed(synth.cbd(g, pr.n), pr.log_n, mods), pr.log_n, mods)
        b = sub_vec(e, mul_vec(a, s_hat, pr.log_n, mods), pr.log_n, mods)
        lo, hi = j * pr.alpha, min((j + 1) * pr.alpha, pr.L)
        if lo < hi:
            gsc = np.array([P % int(mods[t]) if lo <= t < hi else 0 for t in range(kl)], dtype=np.uint64)
            b = add_vec(b, scale_vec(s_from_hat, gsc, pr.log_n, mods), pr.log_n, mods)
        ksk[j, 0] = a
        ksk[j, 1] = b
    return ksk


def rotation_key(pr: Params, s: np.ndarray, gal: int, g: np.random.Generator, seed=None) -> np.ndarray:
    s_hat = secret_eval(pr, s)
    s_rot = automorph(s_hat, pr.log_n, pr.key_mods(), gal, eval_domain=True)
    return switch_key(pr, s_hat, s_rot, g, seed=seed)


def relin_key(pr: Params, s: np.ndarray, g: np.random.Generator) -> np.ndarray:
    s_hat = secret_eval(pr, s)
    s2 = mul_vec(s_hat, s_hat, pr.log_n, pr.key_mods())
    return switch_key(pr, s_hat, s2, g)


def encrypt(pr: Params, s: np.ndarray, m: np.ndarray, level: int, g: np.random.Generator) -> np.ndarray:
    """(a, b) with b = -a*s + m + e over q_0..q_{level-1}, evaluation form."""
    mods = pr.q[:level]
    s_hat = ntt(lift_signed(s, pr.log_n, mods), pr.log_n, mods)
    a = synth.uniform_residues(g, mods, pr.n)
    me = np.asarray(m, dtype=np.int64) + synth.cbd(g, pr.n)
    me_hat = ntt(lift_signed(me, pr.log_n, mods), pr.log_n, mods)
    b = sub_vec(me_hat, mul_vec(a, s_hat, pr.log_n, mods), pr.log_n, mods)
    return np.stack([a, b])


def decrypt_coef(pr: Params, s: np.ndarray, ct: np.ndarray, level: int) -> np.ndarray:
    """coefficient-form residues of a*s + b, [level][N]."""
    mods = pr.q[:level]
    s_hat = ntt(lift_signed(s, pr.log_n, mods), pr.log_n, mods)
    m_hat = add_vec(mul_vec(ct[0], s_hat, pr.log_n, mods), ct[1], pr.log_n, mods)
    return intt(m_hat, pr.log_n, mods)


def centered_small(res: np.ndarray, mods, bound: int):
    """Per coefficient, the integer z with |z| <= bound that every limb agrees on.

    Returns an int64 array, or None if some coefficient's limbs disagree or
    exceed the bound.  Equal small centered residues across coprime moduli
    pin the integer by the Chinese remainder theorem.
    """
    z = None
    for i, m in enumerate(mods):
        m = int(m)
        assert m < (1 << 62)
        c = res[i].astype(np.int64)
        c = np.where(c > m // 2, c - m, c)
        if z is None:
            z = c
        elif not np.array_equal(z, c):
            return None
    if np.max(np.abs(z)) > bound:
        return None
    return z


def ks_noise_bound(pr: Params, level: int, s: np.ndarray) -> int:
    """B_ks = beta*N*(alpha+1)*rho*B_e + (h_s+1)*K, rho = max_j Qt_j / P.

    Derived from the uncorrected ModUp (xhat_j < |I_j| * Qt_j) and the
    floor-style ModDown (error in [0, K)); B_e = 21 for CBD(21).
    """
    P = 1
    for pk in pr.p:
        P *= int(pk)
    rho = 0.0
    for j in range(pr.beta(level)):
        Qt = 1
        for i in range(j * pr.alpha, min((j + 1) * pr.alpha, level)):
            Qt *= int(pr.q[i])
        rho = max(rho, Qt / P)
    hs = int(np.count_nonzero(s))
    return int(np.ceil(pr.beta(level) * pr.n * (pr.alpha + 1) * rho * 21)) + (hs + 1) * pr.K
