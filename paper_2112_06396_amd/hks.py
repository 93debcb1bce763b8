"""Thin ctypes binding of libhks.so (the C ABI declared in include/hks.h).

Argument marshalling only: every computation runs in the HIP library.  Each
function has the C entry point's name and takes torch tensors on the GPU
(dtype torch.uint64 or torch.int64 holding the same bits, contiguous) where
the C call takes device pointers.  The stream is torch's current stream
unless one is given.  A nonzero status raises HksError.

Loading fails loudly (HksUnavailable) when the built library is missing: there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# HKS_LIBRARY may name another build of the same library (e.g. an A/B variant)
LIB_PATH = os.environ.get("HKS_LIBRARY") or os.path.join(_HERE, "libhks.so")

HKS_OK = 0
HKS_EINVAL = -1
HKS_ENOMEM = -2
HKS_EHIP = -3
HKS_EUNSUPPORTED = -4
HKS_ERANGE = -5
HKS_ESCRATCH = -6

HKS_Q_N = 1
HKS_Q_ALPHA = 2
HKS_Q_BETA = 3
HKS_Q_KSK_WORDS = 4
HKS_Q_WORKSPACE_BYTES = 5
HKS_Q_MODULUS = 6
HKS_Q_L = 7
HKS_Q_K = 8
HKS_Q_DNUM = 9
HKS_Q_BATCH_CAP = 10
HKS_Q_NOALLOC_BYTES = 11
HKS_Q_NOALLOC_MAX_BYTES = 12
HKS_NOALLOC_SCRATCH_BYTES = 128 << 20  # the allocation-free scratch (include/hks.h)

# every symbol declared in include/hks.h
EXPORTS = (
    "hks_gen_primes", "hks_galois_for_rotation", "hks_galois_conjugate", "hks_strerror",
    "hks_create", "hks_destroy", "hks_query", "hks_ntt", "hks_intt", "hks_automorph",
    "hks_modup", "hks_ksk_inner", "hks_moddown", "hks_keyswitch", "hks_rotate", "hks_rotate_noalloc",
    "hks_hrotate",
    "hks_batch_rotate", "hks_batch_rotate_mixed", "hks_batch_mult_relin_mixed", "hks_rescale", "hks_ptmult", "hks_mult_relin", "hks_batch_mult_relin", "hks_new_mult",
    "hks_batch_new_mult",
    "hks_encode", "hks_add",
    "hks_expand_key_a", "hks_rotate_seeded", "hks_batch_rotate_seeded", "hks_batch_mult_relin_seeded",
    "hks_ptmatvec", "hks_set_check",
    "hks_get_plan", "hks_set_plan",
    "hks_graph_begin", "hks_graph_end", "hks_graph_launch", "hks_graph_destroy", "hks_prof_enable",
    "hks_prof_read", "hks_modmul_rate",
)

# every symbol declared in include/hks32.h (the 32-bit-word key-switch)
EXPORTS32 = ("hks32_create", "hks32_destroy", "hks32_ntt", "hks32_intt", "hks32_rotate", "hks32_hrotate")

HKS_K_NTT_FWD_COLS = 0
HKS_K_NTT_FWD_ROWS = 1
HKS_K_NTT_INV_ROWS = 2
HKS_K_NTT_INV_COLS = 3
HKS_K_CONV = 4
HKS_K_KSK = 5
HKS_K_MODDOWN_EPI = 6
HKS_K_AUTOMORPH = 7
HKS_K_ELEMENTWISE = 8
HKS_K_NAMES = ("ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols", "conv", "ksk",
               "moddown_epi", "automorph", "elementwise")


class HksError(RuntimeError):
    def __init__(self, name, status):
        super().__init__(f"{name} failed: {status} ({strerror(status)})")
        self.status = status


class HksUnavailable(RuntimeError):
    pass


class _Params(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_uint32),
        ("L", ctypes.c_uint32),
        ("K", ctypes.c_uint32),
        ("dnum", ctypes.c_uint32),
        ("q", ctypes.POINTER(ctypes.c_uint64)),
        ("p", ctypes.POINTER(ctypes.c_uint64)),
        ("max_batch", ctypes.c_uint32),
    ]


class _Plan(ctypes.Structure):
    _fields_ = [
        ("e16_min_waves", ctypes.c_uint32 * 4),
        ("conv_group_limbs", ctypes.c_uint32),
        ("conv_group_max_batch", ctypes.c_uint32),
        ("row_xcd_order", ctypes.c_uint32),
        ("ksk_xcd_order", ctypes.c_uint32),
        ("n1", ctypes.c_uint32),
        ("col_lines", ctypes.c_uint32),
        ("row_lines", ctypes.c_uint32),
    ]


# hks_plan fields as a flat dict: e16_min_waves is split per NTT pass class
PLAN_FIELDS = ("e16_fwd_cols", "e16_fwd_rows", "e16_inv_rows", "e16_inv_cols", "conv_group_limbs",
               "conv_group_max_batch", "row_xcd_order", "ksk_xcd_order", "n1", "col_lines", "row_lines")


class _Params32(ctypes.Structure):
    _fields_ = [
        ("log_n", ctypes.c_uint32),
        ("L", ctypes.c_uint32),
        ("K", ctypes.c_uint32),
        ("dnum", ctypes.c_uint32),
        ("q", ctypes.POINTER(ctypes.c_uint32)),
        ("p", ctypes.POINTER(ctypes.c_uint32)),
    ]


_lib = None
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_i32 = ctypes.c_int


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HksUnavailable(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        sig = {
            "hks_gen_primes": (_i32, [_u32, _u32, _u32, u64p]),
            "hks_galois_for_rotation": (_u32, [ctypes.c_int32, _u32]),
            "hks_galois_conjugate": (_u32, [_u32]),
            "hks_strerror": (ctypes.c_char_p, [_i32]),
            "hks_create": (_i32, [ctypes.POINTER(_Params), _i32, ctypes.POINTER(_vp)]),
            "hks_destroy": (None, [_vp]),
            "hks_query": (_i32, [_vp, _i32, _u32, u64p]),
            "hks_ntt": (_i32, [_vp, _vp, _u32, _u32, _vp]),
            "hks_intt": (_i32, [_vp, _vp, _u32, _u32, _vp]),
            "hks_automorph": (_i32, [_vp, _vp, _vp, _u32, _u32, _u32, _i32, _vp]),
            "hks_modup": (_i32, [_vp, _vp, _u32, _vp, _vp]),
            "hks_ksk_inner": (_i32, [_vp, _vp, _u32, _vp, _vp, _vp]),
            "hks_moddown": (_i32, [_vp, _vp, _u32, _vp, _vp]),
            "hks_keyswitch": (_i32, [_vp, _vp, _u32, _vp, _vp, _vp]),
            "hks_rotate": (_i32, [_vp, _vp, _u32, _u32, _vp, _vp, _vp]),
            "hks_rotate_noalloc": (_i32, [_vp, _vp, _u32, _u32, _vp, _vp, _vp]),
            "hks_hrotate": (_i32, [_vp, _vp, _u32, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_vp),
                                   ctypes.POINTER(_vp), _vp]),
            "hks_batch_rotate": (_i32, [_vp, _u32, ctypes.POINTER(_vp), _u32, ctypes.POINTER(_u32),
                                        ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
            "hks_batch_rotate_mixed": (_i32, [_vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_u32),
                                              ctypes.POINTER(_u32), u64p, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                              _vp]),
            "hks_batch_mult_relin_mixed": (_i32, [_vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                  ctypes.POINTER(_u32), u64p, ctypes.POINTER(_vp), _i32,
                                                  ctypes.POINTER(_vp), _vp]),
            "hks_rescale": (_i32, [_vp, _vp, _u32, _vp, _vp]),
            "hks_ptmult": (_i32, [_vp, _vp, _vp, _u32, _i32, _vp, _vp]),
            "hks_mult_relin": (_i32, [_vp, _vp, _vp, _u32, _vp, _i32, _vp, _vp]),
            "hks_batch_mult_relin": (_i32, [_vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u32,
                                            ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), _vp]),
            "hks_new_mult": (_i32, [_vp, _vp, _vp, _u32, _vp, _vp, _vp]),
            "hks_batch_new_mult": (_i32, [_vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u32,
                                          ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
            "hks_encode": (_i32, [_vp, _vp, ctypes.c_double, _u32, _i32, _vp, _vp]),
            "hks_add": (_i32, [_vp, _vp, _vp, _u32, _u32, _vp, _vp]),
            "hks_expand_key_a": (_i32, [_vp, ctypes.c_uint64, _vp, _vp]),
            "hks_ptmatvec": (_i32, [_vp, _vp, _u32, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_vp),
                                    ctypes.POINTER(_vp), _vp, _vp]),
            "hks_rotate_seeded": (_i32, [_vp, _vp, _u32, _u32, ctypes.c_uint64, _vp, _vp, _vp]),
            "hks_batch_rotate_seeded": (_i32, [_vp, _u32, ctypes.POINTER(_vp), _u32, ctypes.POINTER(_u32), u64p,
                                               ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp]),
            "hks_batch_mult_relin_seeded": (_i32, [_vp, _u32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _u32, u64p,
                                                   ctypes.POINTER(_vp), _i32, ctypes.POINTER(_vp), _vp]),
            "hks_set_check": (_i32, [_vp, _i32]),
            "hks_get_plan": (_i32, [_vp, ctypes.POINTER(_Plan)]),
            "hks_set_plan": (_i32, [_vp, ctypes.POINTER(_Plan)]),
            "hks_graph_begin": (_i32, [_vp]),
            "hks_graph_end": (_i32, [_vp, ctypes.POINTER(_vp)]),
            "hks_graph_launch": (_i32, [_vp, _vp]),
            "hks_graph_destroy": (None, [_vp]),
            "hks32_create": (_i32, [ctypes.POINTER(_Params32), _i32, ctypes.POINTER(_vp)]),
            "hks32_destroy": (None, [_vp]),
            "hks32_ntt": (_i32, [_vp, _vp, _u32, _u32, _vp]),
            "hks32_intt": (_i32, [_vp, _vp, _u32, _u32, _vp]),
            "hks32_rotate": (_i32, [_vp, _vp, _u32, _u32, _vp, _vp, _vp]),
            "hks32_hrotate": (_i32, [_vp, _vp, _u32, _u32, ctypes.POINTER(_u32), ctypes.POINTER(_vp),
                                     ctypes.POINTER(_vp), _vp]),
            "hks_prof_enable": (_i32, [_vp, _u32]),
            "hks_prof_read": (_i32, [_vp, _i32, ctypes.POINTER(ctypes.c_double), u64p]),
            "hks_modmul_rate": (_i32, [_vp, _u32, _vp, ctypes.POINTER(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().hks_strerror(int(status)).decode()


def _check(name, rc):
    if rc != HKS_OK:
        raise HksError(name, rc)


def _on_device(t: torch.Tensor) -> bool:
    return t.is_cuda


class HksSizeError(ValueError):
    """A tensor holds fewer words than the call reads or writes through it."""


def _need(t, words: int, what: str):
    if words is not None and t.numel() < words:
        raise HksSizeError(f"{what}: {t.numel()} words, the call touches {words}")


def _ptr(t: torch.Tensor, words: int = None, what: str = "tensor"):
    """Device pointer of t, after checking its dtype, that it holds at least
    `words` words (the extent the C call reads or writes), and that it is a
    contiguous GPU tensor."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype not in (torch.uint64, torch.int64):
        raise TypeError(f"expected 64-bit integer tensor, got {t.dtype}")
    _need(t, words, what)
    if not _on_device(t):
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


# Words a call touches through each argument (layouts of include/hks.h).  A
# level outside [1, L] is left to the C call, which rejects it.
def _lvl(ctx, level):
    return int(level) if 1 <= int(level) <= ctx.L else None


def _w_poly(ctx, level, polys=1):
    lv = _lvl(ctx, level)
    return None if lv is None else polys * lv * ctx.n


def _w_ext(ctx, level):
    """one polynomial over Q_level U P"""
    lv = _lvl(ctx, level)
    return None if lv is None else (lv + ctx.K) * ctx.n


def _w_digits(ctx, level):
    """the extended digits [beta][level + K][N]"""
    lv = _lvl(ctx, level)
    if lv is None:
        return None
    alpha = -(-ctx.L // ctx.dnum)
    return -(-lv // alpha) * (lv + ctx.K) * ctx.n


def _w_key(ctx):
    """a switching key [dnum][2][L + K][N]"""
    return ctx.dnum * 2 * (ctx.L + ctx.K) * ctx.n


def _w_key_rows(ctx):
    """one row per digit, [dnum][L + K][N] (a seeded key's b_j, or its a_j)"""
    return ctx.dnum * (ctx.L + ctx.K) * ctx.n


def _w_out(ctx, level, drop):
    """a ciphertext [2][level - drop][N] (drop = 1 after a Rescale)"""
    lv = _lvl(ctx, level)
    return None if lv is None or lv - drop < 1 else 2 * (lv - drop) * ctx.n


def _w_limbs(ctx, first_mod, n_limbs):
    if first_mod + n_limbs > ctx.L + ctx.K:
        return None
    return n_limbs * ctx.n


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


# ---------------------------------------------------------------- host helpers

def hks_gen_primes(bits: int, log_step: int, count: int):
    out = (ctypes.c_uint64 * count)()
    _check("hks_gen_primes", lib().hks_gen_primes(bits, log_step, count, out))
    return [int(v) for v in out]


def hks_galois_for_rotation(k: int, log_n: int) -> int:
    return int(lib().hks_galois_for_rotation(int(k), int(log_n)))


def hks_galois_conjugate(log_n: int) -> int:
    return int(lib().hks_galois_conjugate(int(log_n)))


def hks_strerror(status: int) -> str:
    return strerror(status)


# ---------------------------------------------------------------- context

class Context:
    """Owns an hks_ctx (tables + workspace on one device)."""

    def __init__(self, log_n: int, q, p, dnum: int, device: int = 0, max_batch: int = 1):
        self.q = [int(v) for v in q]
        self.p = [int(v) for v in p]
        self.log_n, self.L, self.K, self.dnum = int(log_n), len(self.q), len(self.p), int(dnum)
        qa = (ctypes.c_uint64 * self.L)(*self.q)
        pa = (ctypes.c_uint64 * self.K)(*self.p)
        prm = _Params(self.log_n, self.L, self.K, self.dnum, qa, pa, int(max_batch))
        h = ctypes.c_void_p()
        _check("hks_create", lib().hks_create(ctypes.byref(prm), int(device), ctypes.byref(h)))
        self._h = h
        self.n = 1 << self.log_n
        self.alpha = -(-self.L // self.dnum)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context destroyed")
        return self._h

    def query(self, key: int, level: int = 0) -> int:
        return hks_query(self, key, level)

    def beta(self, level: int) -> int:
        return -(-level // self.alpha)

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().hks_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def hks_create(log_n: int, q, p, dnum: int, device: int = 0) -> Context:
    return Context(log_n, q, p, dnum, device)


def hks_destroy(ctx: Context) -> None:
    ctx.close()


def hks_query(ctx: Context, key: int, level: int = 0) -> int:
    out = ctypes.c_uint64()
    _check("hks_query", lib().hks_query(ctx.handle, int(key), int(level), ctypes.byref(out)))
    return int(out.value)


# ---------------------------------------------------------------- calls

def hks_ntt(ctx, x, first_mod: int, n_limbs: int, stream=None):
    _check("hks_ntt", lib().hks_ntt(ctx.handle, _ptr(x, _w_limbs(ctx, first_mod, n_limbs), "x"), first_mod,
                                    n_limbs, _stream(stream)))


def hks_intt(ctx, x, first_mod: int, n_limbs: int, stream=None):
    _check("hks_intt", lib().hks_intt(ctx.handle, _ptr(x, _w_limbs(ctx, first_mod, n_limbs), "x"), first_mod,
                                      n_limbs, _stream(stream)))


def hks_automorph(ctx, x, y, first_mod: int, n_limbs: int, galois: int, eval_domain: bool = True, stream=None):
    w = _w_limbs(ctx, first_mod, n_limbs)
    _check("hks_automorph", lib().hks_automorph(ctx.handle, _ptr(x, w, "x"), _ptr(y, w, "y"), first_mod, n_limbs, galois,
                                                1 if eval_domain else 0, _stream(stream)))


def hks_modup(ctx, a, level: int, ext, stream=None):
    _check("hks_modup", lib().hks_modup(ctx.handle, _ptr(a, _w_poly(ctx, level), "a"), level,
                                        _ptr(ext, _w_digits(ctx, level), "ext"), _stream(stream)))


def hks_ksk_inner(ctx, ext, level: int, ksk, uv, stream=None):
    _check("hks_ksk_inner", lib().hks_ksk_inner(ctx.handle, _ptr(ext, _w_digits(ctx, level), "ext"), level,
                                                _ptr(ksk, _w_key(ctx), "ksk"), _ptr(uv, 2 * (_w_ext(ctx, level) or 0) or None, "uv"),
                                                _stream(stream)))


def hks_moddown(ctx, x, level: int, y, stream=None):
    _check("hks_moddown", lib().hks_moddown(ctx.handle, _ptr(x, _w_ext(ctx, level), "x"), level,
                                            _ptr(y, _w_poly(ctx, level), "y"), _stream(stream)))


def hks_keyswitch(ctx, d, level: int, ksk, uv, stream=None):
    _check("hks_keyswitch", lib().hks_keyswitch(ctx.handle, _ptr(d, _w_poly(ctx, level), "d"), level,
                                                _ptr(ksk, _w_key(ctx), "ksk"), _ptr(uv, _w_poly(ctx, level, 2), "uv"),
                                                _stream(stream)))


def hks_rotate(ctx, ct, level: int, galois: int, ksk, ct_out, stream=None):
    _check("hks_rotate", lib().hks_rotate(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"), level, galois,
                                          _ptr(ksk, _w_key(ctx), "ksk"), _ptr(ct_out, _w_poly(ctx, level, 2), "ct_out"),
                                          _stream(stream)))


def hks_rotate_noalloc(ctx, ct, level: int, galois: int, ksk, ct_out, stream=None):
    _check("hks_rotate_noalloc",
           lib().hks_rotate_noalloc(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"), level, galois,
                                    _ptr(ksk, _w_key(ctx), "ksk"), _ptr(ct_out, _w_poly(ctx, level, 2), "ct_out"),
                                    _stream(stream)))


def hks_hrotate(ctx, ct, level: int, galois, ksks, outs, stream=None):
    r = len(galois)
    if len(ksks) != r or len(outs) != r:
        raise ValueError("galois, ksks and outs must have the same length")
    ga = (_u32 * r)(*[int(g) for g in galois])
    ka = (_vp * r)(*[_ptr(k, _w_key(ctx), "ksk") for k in ksks])
    oa = (_vp * r)(*[_ptr(o, _w_poly(ctx, level, 2), "ct_out") for o in outs])
    _check("hks_hrotate", lib().hks_hrotate(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"), level, r, ga, ka, oa,
                                            _stream(stream)))


def hks_batch_rotate(ctx, cts, level: int, galois, ksks, outs, stream=None):
    n = len(cts)
    if len(galois) != n or len(ksks) != n or len(outs) != n:
        raise ValueError("cts, galois, ksks and outs must have the same length")
    ca = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct") for c in cts])
    ga = (_u32 * n)(*[int(g) for g in galois])
    ka = (_vp * n)(*[_ptr(k, _w_key(ctx), "ksk") for k in ksks])
    oa = (_vp * n)(*[_ptr(o, _w_poly(ctx, level, 2), "ct_out") for o in outs])
    _check("hks_batch_rotate", lib().hks_batch_rotate(ctx.handle, n, ca, level, ga, ka, oa, _stream(stream)))


def hks_rescale(ctx, ct, level: int, ct_out, stream=None):
    _check("hks_rescale", lib().hks_rescale(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"), level,
                                            _ptr(ct_out, _w_out(ctx, level, 1), "ct_out"), _stream(stream)))


def hks_ptmult(ctx, ct, pt, level: int, rescale: bool, ct_out, stream=None):
    _check("hks_ptmult", lib().hks_ptmult(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"),
                                          _ptr(pt, _w_poly(ctx, level), "pt"), level, 1 if rescale else 0,
                                          _ptr(ct_out, _w_out(ctx, level, 1 if rescale else 0), "ct_out"),
                                          _stream(stream)))


def hks_batch_mult_relin(ctx, ct1s, ct2s, level: int, rlks, rescale: bool, outs, stream=None):
    n = len(ct1s)
    if len(ct2s) != n or len(rlks) != n or len(outs) != n:
        raise ValueError("ct1s, ct2s, rlks and outs must have the same length")
    a = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct1") for c in ct1s])
    b = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct2") for c in ct2s])
    k = (_vp * n)(*[_ptr(r, _w_key(ctx), "rlk") for r in rlks])
    o = (_vp * n)(*[_ptr(x, _w_out(ctx, level, 1 if rescale else 0), "ct_out") for x in outs])
    _check("hks_batch_mult_relin", lib().hks_batch_mult_relin(ctx.handle, n, a, b, level, k, 1 if rescale else 0, o,
                                                              _stream(stream)))


def hks_batch_new_mult(ctx, ct1s, ct2s, level: int, rlks, outs, stream=None):
    n = len(ct1s)
    if len(ct2s) != n or len(rlks) != n or len(outs) != n:
        raise ValueError("ct1s, ct2s, rlks and outs must have the same length")
    a = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct1") for c in ct1s])
    b = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct2") for c in ct2s])
    k = (_vp * n)(*[_ptr(r, _w_key(ctx), "rlk") for r in rlks])
    o = (_vp * n)(*[_ptr(x, _w_out(ctx, level, 1), "ct_out") for x in outs])
    _check("hks_batch_new_mult", lib().hks_batch_new_mult(ctx.handle, n, a, b, level, k, o, _stream(stream)))


def hks_batch_rotate_mixed(ctx, cts, levels, galois, ksks, outs, seeds=None, stream=None):
    """Rotate of ciphertexts at uneven levels in shared launches; seeds given:
    ksks[i] holds the rows b_j of seeded key seeds[i]."""
    n = len(cts)
    if len(levels) != n or len(galois) != n or len(ksks) != n or len(outs) != n or (seeds is not None
                                                                                     and len(seeds) != n):
        raise ValueError("cts, levels, galois, ksks, outs (and seeds) must have the same length")
    ca = (_vp * n)(*[_ptr(c, _w_poly(ctx, lv, 2), "ct") for c, lv in zip(cts, levels)])
    la = (_u32 * n)(*[int(lv) for lv in levels])
    ga = (_u32 * n)(*[int(g) for g in galois])
    sa = None if seeds is None else (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    kw = _w_key(ctx) if seeds is None else _w_key_rows(ctx)
    ka = (_vp * n)(*[_ptr(k, kw, "ksk") for k in ksks])
    oa = (_vp * n)(*[_ptr(o, _w_poly(ctx, lv, 2), "ct_out") for o, lv in zip(outs, levels)])
    _check("hks_batch_rotate_mixed", lib().hks_batch_rotate_mixed(ctx.handle, n, ca, la, ga, sa, ka, oa,
                                                                  _stream(stream)))


def hks_batch_mult_relin_mixed(ctx, ct1s, ct2s, levels, rlks, rescale: bool, outs, seeds=None, stream=None):
    """Mult + relinearization of pairs at uneven levels in shared launches."""
    n = len(ct1s)
    if len(ct2s) != n or len(levels) != n or len(rlks) != n or len(outs) != n or (seeds is not None
                                                                                  and len(seeds) != n):
        raise ValueError("ct1s, ct2s, levels, rlks, outs (and seeds) must have the same length")
    a = (_vp * n)(*[_ptr(c, _w_poly(ctx, lv, 2), "ct1") for c, lv in zip(ct1s, levels)])
    b = (_vp * n)(*[_ptr(c, _w_poly(ctx, lv, 2), "ct2") for c, lv in zip(ct2s, levels)])
    la = (_u32 * n)(*[int(lv) for lv in levels])
    sa = None if seeds is None else (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    kw = _w_key(ctx) if seeds is None else _w_key_rows(ctx)
    k = (_vp * n)(*[_ptr(r, kw, "rlk") for r in rlks])
    o = (_vp * n)(*[_ptr(x, _w_out(ctx, lv, 1 if rescale else 0), "ct_out") for x, lv in zip(outs, levels)])
    _check("hks_batch_mult_relin_mixed", lib().hks_batch_mult_relin_mixed(ctx.handle, n, a, b, la, sa, k,
                                                                          1 if rescale else 0, o, _stream(stream)))


def hks_ptmatvec(ctx, ct, level: int, galois, ksks, pts, ct_out, stream=None):
    """ksks[i] = None (with galois[i] = 1): the diagonal without rotation."""
    r = len(galois)
    if len(ksks) != r or len(pts) != r:
        raise ValueError("galois, ksks and pts must have the same length")
    ga = (_u32 * r)(*[int(g) for g in galois])
    ka = (_vp * r)(*[_vp() if k is None else _ptr(k, _w_key(ctx), "ksk") for k in ksks])
    pa = (_vp * r)(*[_ptr(p, _w_ext(ctx, level), "pt") for p in pts])
    _check("hks_ptmatvec", lib().hks_ptmatvec(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"), level, r, ga, ka,
                                              pa, _ptr(ct_out, _w_poly(ctx, level, 2), "ct_out"), _stream(stream)))


def hks_expand_key_a(ctx, seed: int, a, stream=None):
    _check("hks_expand_key_a", lib().hks_expand_key_a(ctx.handle, int(seed), _ptr(a, _w_key_rows(ctx), "a"),
                                                      _stream(stream)))


def hks_rotate_seeded(ctx, ct, level: int, galois: int, seed: int, ksk_b, ct_out, stream=None):
    _check("hks_rotate_seeded", lib().hks_rotate_seeded(ctx.handle, _ptr(ct, _w_poly(ctx, level, 2), "ct"), level,
                                                        galois, int(seed), _ptr(ksk_b, _w_key_rows(ctx), "ksk_b"),
                                                        _ptr(ct_out, _w_poly(ctx, level, 2), "ct_out"),
                                                        _stream(stream)))


def hks_batch_rotate_seeded(ctx, cts, level: int, galois, seeds, ksk_bs, outs, stream=None):
    n = len(cts)
    if len(galois) != n or len(seeds) != n or len(ksk_bs) != n or len(outs) != n:
        raise ValueError("cts, galois, seeds, ksk_bs and outs must have the same length")
    ca = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct") for c in cts])
    ga = (_u32 * n)(*[int(g) for g in galois])
    sa = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    ka = (_vp * n)(*[_ptr(k, _w_key_rows(ctx), "ksk_b") for k in ksk_bs])
    oa = (_vp * n)(*[_ptr(o, _w_poly(ctx, level, 2), "ct_out") for o in outs])
    _check("hks_batch_rotate_seeded", lib().hks_batch_rotate_seeded(ctx.handle, n, ca, level, ga, sa, ka, oa,
                                                                    _stream(stream)))


def hks_batch_mult_relin_seeded(ctx, ct1s, ct2s, level: int, seeds, rlk_bs, rescale: bool, outs, stream=None):
    n = len(ct1s)
    if len(ct2s) != n or len(seeds) != n or len(rlk_bs) != n or len(outs) != n:
        raise ValueError("ct1s, ct2s, seeds, rlk_bs and outs must have the same length")
    a1 = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct1") for c in ct1s])
    a2 = (_vp * n)(*[_ptr(c, _w_poly(ctx, level, 2), "ct2") for c in ct2s])
    sa = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    ka = (_vp * n)(*[_ptr(k, _w_key_rows(ctx), "rlk_b") for k in rlk_bs])
    oa = (_vp * n)(*[_ptr(o, _w_out(ctx, level, 1 if rescale else 0), "ct_out") for o in outs])
    _check("hks_batch_mult_relin_seeded", lib().hks_batch_mult_relin_seeded(ctx.handle, n, a1, a2, level, sa, ka,
                                                                            1 if rescale else 0, oa, _stream(stream)))


def hks_new_mult(ctx, ct1, ct2, level: int, rlk, ct_out, stream=None):
    _check("hks_new_mult", lib().hks_new_mult(ctx.handle, _ptr(ct1, _w_poly(ctx, level, 2), "ct1"),
                                              _ptr(ct2, _w_poly(ctx, level, 2), "ct2"), level,
                                              _ptr(rlk, _w_key(ctx), "rlk"), _ptr(ct_out, _w_out(ctx, level, 1), "ct_out"),
                                              _stream(stream)))


def hks_encode(ctx, slots, scale: float, level: int, with_p: bool, pt_out, stream=None):
    """slots: complex128 (or float64 [.., 2]) device tensor of N/2 values."""
    if slots.dtype == torch.complex128:
        slots = torch.view_as_real(slots)
    if slots.dtype != torch.float64 or not slots.is_cuda or not slots.is_contiguous():
        raise ValueError("slots must be a contiguous complex128/float64 device tensor")
    if slots.numel() != ctx.n:
        raise ValueError("expected N/2 complex slots")
    w = _w_ext(ctx, level) if with_p else _w_poly(ctx, level)
    _check("hks_encode", lib().hks_encode(ctx.handle, ctypes.c_void_p(slots.data_ptr()), float(scale), level,
                                          1 if with_p else 0, _ptr(pt_out, w, "pt_out"), _stream(stream)))


def hks_set_check(ctx, on: bool):
    _check("hks_set_check", lib().hks_set_check(ctx.handle, 1 if on else 0))


def hks_get_plan(ctx) -> dict:
    """The context's launch plan as a flat dict (keys PLAN_FIELDS)."""
    p = _Plan()
    _check("hks_get_plan", lib().hks_get_plan(ctx.handle, ctypes.byref(p)))
    vals = list(p.e16_min_waves) + [p.conv_group_limbs, p.conv_group_max_batch, p.row_xcd_order, p.ksk_xcd_order,
                                    p.n1, p.col_lines, p.row_lines]
    return dict(zip(PLAN_FIELDS, (int(v) for v in vals)))


def hks_set_plan(ctx, plan: dict):
    """Sets the launch plan from a flat dict (keys PLAN_FIELDS; missing keys
    keep the context's current values)."""
    cur = hks_get_plan(ctx)
    unknown = set(plan) - set(PLAN_FIELDS)
    if unknown:
        raise ValueError(f"unknown plan fields {sorted(unknown)}")
    cur.update({k: int(v) for k, v in plan.items()})
    p = _Plan()
    for i, k in enumerate(PLAN_FIELDS[:4]):
        p.e16_min_waves[i] = cur[k]
    p.conv_group_limbs, p.conv_group_max_batch = cur["conv_group_limbs"], cur["conv_group_max_batch"]
    p.row_xcd_order, p.ksk_xcd_order = cur["row_xcd_order"], cur["ksk_xcd_order"]
    p.n1, p.col_lines, p.row_lines = cur["n1"], cur["col_lines"], cur["row_lines"]
    _check("hks_set_plan", lib().hks_set_plan(ctx.handle, ctypes.byref(p)))


class Graph:
    """A call sequence recorded on a stream and replayed as one HIP graph."""

    def __init__(self, handle):
        self._h = handle

    def launch(self, stream):
        _check("hks_graph_launch", lib().hks_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().hks_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hks_graph_begin(stream):
    _check("hks_graph_begin", lib().hks_graph_begin(_stream(stream)))


def hks_graph_end(stream) -> Graph:
    h = ctypes.c_void_p()
    _check("hks_graph_end", lib().hks_graph_end(_stream(stream), ctypes.byref(h)))
    return Graph(h)


def hks_add(ctx, x, y, level: int, n_poly: int, out, stream=None):
    w = _w_poly(ctx, level, int(n_poly)) if 1 <= int(n_poly) <= 3 else None
    _check("hks_add", lib().hks_add(ctx.handle, _ptr(x, w, "x"), _ptr(y, w, "y"), level, n_poly, _ptr(out, w, "out"),
                                    _stream(stream)))


def hks_mult_relin(ctx, ct1, ct2, level: int, rlk, rescale: bool, ct_out, stream=None):
    _check("hks_mult_relin", lib().hks_mult_relin(ctx.handle, _ptr(ct1, _w_poly(ctx, level, 2), "ct1"),
                                                  _ptr(ct2, _w_poly(ctx, level, 2), "ct2"), level,
                                                  _ptr(rlk, _w_key(ctx), "rlk"), 1 if rescale else 0,
                                                  _ptr(ct_out, _w_out(ctx, level, 1 if rescale else 0), "ct_out"),
                                                  _stream(stream)))


def hks_prof_enable(ctx, mask: int):
    _check("hks_prof_enable", lib().hks_prof_enable(ctx.handle, int(mask)))


def hks_prof_read(ctx, kernel_class: int):
    """(milliseconds summed over launches, launch count) for one kernel class."""
    ms = ctypes.c_double()
    n = ctypes.c_uint64()
    _check("hks_prof_read", lib().hks_prof_read(ctx.handle, int(kernel_class), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def hks_modmul_rate(ctx, iters: int = 1024, stream=None) -> float:
    """Measured lazy Shoup products per second (uses the context's workspace)."""
    r = ctypes.c_double()
    _check("hks_modmul_rate", lib().hks_modmul_rate(ctx.handle, int(iters), _stream(stream), ctypes.byref(r)))
    return float(r.value)


# ---------------------------------------------------------------- tensor helpers

class Context32:
    """Owns an hks32_ctx: the key-switch in 32-bit words (primes below 2^30)."""

    def __init__(self, log_n: int, q, p, dnum: int, device: int = 0):
        self.q = [int(v) for v in q]
        self.p = [int(v) for v in p]
        self.log_n, self.L, self.K, self.dnum = int(log_n), len(self.q), len(self.p), int(dnum)
        qa = (ctypes.c_uint32 * self.L)(*self.q)
        pa = (ctypes.c_uint32 * self.K)(*self.p)
        prm = _Params32(self.log_n, self.L, self.K, self.dnum, qa, pa)
        h = ctypes.c_void_p()
        _check("hks32_create", lib().hks32_create(ctypes.byref(prm), int(device), ctypes.byref(h)))
        self._h = h
        self.n = 1 << self.log_n

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context destroyed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().hks32_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr32(t: torch.Tensor, words: int = None, what: str = "tensor"):
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"expected 32-bit integer tensor, got {t.dtype}")
    _need(t, words, what)
    if not _on_device(t) or not t.is_contiguous():
        raise ValueError("tensor must be a contiguous GPU tensor")
    return ctypes.c_void_p(t.data_ptr())


def hks32_ntt(ctx, x, first_mod: int, n_limbs: int, stream=None):
    _check("hks32_ntt", lib().hks32_ntt(ctx.handle, _ptr32(x, _w_limbs(ctx, first_mod, n_limbs), "x"), first_mod,
                                        n_limbs, _stream(stream)))


def hks32_intt(ctx, x, first_mod: int, n_limbs: int, stream=None):
    _check("hks32_intt", lib().hks32_intt(ctx.handle, _ptr32(x, _w_limbs(ctx, first_mod, n_limbs), "x"), first_mod,
                                          n_limbs, _stream(stream)))


def hks32_rotate(ctx, ct, level: int, galois: int, ksk, ct_out, stream=None):
    _check("hks32_rotate", lib().hks32_rotate(ctx.handle, _ptr32(ct, _w_poly(ctx, level, 2), "ct"), level, galois,
                                              _ptr32(ksk, _w_key(ctx), "ksk"),
                                              _ptr32(ct_out, _w_poly(ctx, level, 2), "ct_out"), _stream(stream)))


def hks32_hrotate(ctx, ct, level: int, galois, ksks, outs, stream=None):
    r = len(galois)
    if len(ksks) != r or len(outs) != r:
        raise ValueError("galois, ksks and outs must have the same length")
    ga = (_u32 * r)(*[int(g) for g in galois])
    ka = (_vp * r)(*[_ptr32(k, _w_key(ctx), "ksk") for k in ksks])
    oa = (_vp * r)(*[_ptr32(o, _w_poly(ctx, level, 2), "ct_out") for o in outs])
    _check("hks32_hrotate", lib().hks32_hrotate(ctx.handle, _ptr32(ct, _w_poly(ctx, level, 2), "ct"), level, r, ga,
                                                ka, oa, _stream(stream)))


def to_device32(a, device="cuda") -> torch.Tensor:
    """numpy array of residues below 2^32 -> contiguous int32 GPU tensor (bit copy)."""
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a).astype(np.uint32))
    return torch.from_numpy(a.view(np.int32)).to(device)


def to_host32(t: torch.Tensor):
    """32-bit GPU tensor -> numpy uint64 array of the same residues."""
    import numpy as np
    return t.view(torch.int32).cpu().numpy().view(np.uint32).astype(np.uint64)


def empty32(shape, device="cuda") -> torch.Tensor:
    return torch.empty(shape, dtype=torch.int32, device=device)


def to_device(a, device="cuda") -> torch.Tensor:
    """numpy uint64 array -> contiguous torch.uint64 tensor on the GPU (bit copy)."""
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device).view(torch.uint64)


def to_host(t: torch.Tensor):
    """GPU tensor -> numpy uint64 array (bit copy)."""
    import numpy as np
    return t.view(torch.int64).cpu().numpy().view(np.uint64)


def empty(shape, device="cuda") -> torch.Tensor:
    return torch.empty(shape, dtype=torch.int64, device=device).view(torch.uint64)
