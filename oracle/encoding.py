"""CKKS encoding and the factored homomorphic DFT of bootstrapping's linear
layers (test infrastructure only, like the rest of ``oracle/``).

Slots.  For a real polynomial m of degree < N, slot j (j < n = N/2) is
m(zeta^(g_j)) with zeta = exp(i pi / N) and g_j = 5^j mod 2N (the rotation
group; rotating the slots right by k is the automorphism X -> X^(5^-k)).
Writing w_k = m_k + i m_(k+n) (k < n) and using zeta^(g_j n) = i (g_j = 1
mod 4), the slot vector is z = V w with V[j, k] = zeta^(g_j k), an n x n
matrix with V^H V = n I.  So decoding is z = V w and encoding is
w = V^H z / n, then m = round(Delta * (Re w, Im w)).

Factored DFT (Sec. 3, bootstrapping's CoeffToSlot / SlotToCoeff).  Splitting
w into even and odd indices gives, for j < m/2 in a block of size m,
z_j = E_j + w_m(j) O_j and z_(j+m/2) = E_j - w_m(j) O_j with
w_m(j) = exp(2 pi i (5^j mod 4m) / (4m)), so
    V = S_n S_(n/2) ... S_2 R
with R the bit-reversal permutation and S_m the block-diagonal butterfly
stage of block size m.  Each S_m has three non-zero generalized diagonals
(offsets 0, +m/2, -m/2 of the cyclic slot index).  A matrix in diagonal form
is {d: D_d} with (A x)_j = sum_d D_d[j] x_((j - d) mod n): the term d is the
diagonal D_d times the slots rotated right by d.  SlotToCoeff applies
S_2, ..., S_n to R w; CoeffToSlot applies S_n^-1, ..., S_2^-1 to z and
leaves R w.  fftIter groups of consecutive stages are multiplied out; the
number of stages per group is balanced with the larger groups last (the
paper's rule for the radices), and a group of r stages has at most
2^(r+1) - 1 diagonals.

Everything here is numpy float64/complex128; numpy's FFT serves as the one
library step of encode/decode (a length-n DFT over the index t_j with
g_j = 4 t_j + 1).
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def rot_group(n: int) -> np.ndarray:
    """g_j = 5^j mod 4n for j < n (4n = 2N)."""
    g = np.empty(n, dtype=np.int64)
    x = 1
    for j in range(n):
        g[j] = x
        x = (x * 5) % (4 * n)
    return g


def _t_index(n: int) -> np.ndarray:
    """t_j with g_j = 4 t_j + 1; a permutation of 0..n-1."""
    return (rot_group(n) - 1) // 4


def decode_w(w: np.ndarray) -> np.ndarray:
    """z = V w: z_j = sum_k w_k zeta^(g_j k) = n * ifft(w_k zeta^k)[t_j]."""
    w = np.asarray(w, dtype=np.complex128)
    n = len(w)
    zeta = np.exp(1j * np.pi * np.arange(n) / (2 * n))
    return n * np.fft.ifft(w * zeta)[_t_index(n)]


def encode_w(z: np.ndarray) -> np.ndarray:
    """w = V^H z / n: (V^H z)_k = zeta^(-k) sum_j z_j exp(-2 pi i t_j k / n)."""
    z = np.asarray(z, dtype=np.complex128)
    n = len(z)
    Z = np.empty(n, dtype=np.complex128)
    Z[_t_index(n)] = z
    zeta_inv = np.exp(-1j * np.pi * np.arange(n) / (2 * n))
    return zeta_inv * np.fft.fft(Z) / n


def encode(z: np.ndarray, scale: float) -> np.ndarray:
    """Integer coefficients (int64, length N = 2n) of the plaintext whose slots
    are z at scale Delta: round(Delta Re w), round(Delta Im w), half to even."""
    w = encode_w(z) * scale
    return np.concatenate([np.rint(w.real), np.rint(w.imag)]).astype(np.int64)


def decode(m, scale: float) -> np.ndarray:
    """Slots of the real polynomial with coefficients m (numbers; python ints
    allowed) divided by Delta."""
    m = np.asarray([float(v) for v in m], dtype=np.float64)
    n = len(m) // 2
    return decode_w(m[:n] + 1j * m[n:]) / scale


def vandermonde(n: int) -> np.ndarray:
    """The dense V[j, k] = zeta^(g_j k) (closed form, for checks at small n)."""
    g = rot_group(n)
    k = np.arange(n)
    return np.exp(2j * np.pi * np.outer(g, k) / (4 * n))


def bit_reverse_perm(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    return np.array([int(format(i, f"0{bits}b")[::-1], 2) if bits else 0 for i in range(n)], dtype=np.int64)


# --------------------------------------------------------------- diagonal form

def stage(n: int, m: int, inverse: bool) -> dict:
    """S_m (or S_m^-1) in diagonal form.  Rows r = b m + j, j < m/2:
    S_m:    y_r = x_r + w x_(r+m/2),        y_(r+m/2) = x_r - w x_(r+m/2);
    S_m^-1: y_r = (x_r + x_(r+m/2)) / 2,    y_(r+m/2) = w^-1 (x_r - x_(r+m/2)) / 2."""
    h = m // 2
    j = np.arange(n) % m
    top = j < h
    jj = np.where(top, j, j - h)
    g = np.array([pow(5, t, 4 * m) for t in range(h)], dtype=np.int64)  # 5^j mod 4m
    w = np.exp(2j * np.pi * g[jj] / (4 * m))
    d0 = np.empty(n, dtype=np.complex128)
    dm = np.zeros(n, dtype=np.complex128)  # offset -h: row r reads x_(r+h)
    dp = np.zeros(n, dtype=np.complex128)  # offset +h: row r+h reads x_r
    if not inverse:
        d0[top] = 1.0
        dm[top] = w[top]
        d0[~top] = -w[~top]
        dp[~top] = 1.0
    else:
        d0[top] = 0.5
        dm[top] = 0.5
        d0[~top] = -0.5 / w[~top]
        dp[~top] = 0.5 / w[~top]
    out = {0: d0}
    for off, d in ((-h % n, dm), (h % n, dp)):
        out[off] = out.get(off, 0) + d
    return out


def matmul_diag(A: dict, B: dict, n: int) -> dict:
    """A B in diagonal form: C_(a+b)[j] += A_a[j] B_b[j - a]."""
    C = {}
    for a, Da in A.items():
        for b, Db in B.items():
            c = (a + b) % n
            C[c] = C.get(c, 0) + Da * np.roll(Db, a)
    return C


def apply_diag(A: dict, x: np.ndarray) -> np.ndarray:
    """(A x)_j = sum_d A_d[j] x_(j - d)."""
    y = np.zeros(len(x), dtype=np.complex128)
    for d, D in A.items():
        y += D * np.roll(x, d)
    return y


def to_dense(A: dict, n: int) -> np.ndarray:
    M = np.zeros((n, n), dtype=np.complex128)
    r = np.arange(n)
    for d, D in A.items():
        M[r, (r - d) % n] += D
    return M


def radices(log_slots: int, iters: int) -> list:
    """Stages per group: balanced, the larger ones last."""
    base, extra = divmod(log_slots, iters)
    return [base] * (iters - extra) + [base + 1] * extra


def _groups(n: int, iters: int, inverse: bool) -> list:
    logn = n.bit_length() - 1
    ms = [1 << s for s in range(1, logn + 1)]  # S_2 .. S_n, SlotToCoeff's order
    if inverse:
        ms = ms[::-1]  # CoeffToSlot applies S_n^-1 first
    out, pos = [], 0
    for r in radices(logn, iters):
        G = {0: np.ones(n, dtype=np.complex128)}
        for m in ms[pos:pos + r]:
            G = matmul_diag(stage(n, m, inverse), G, n)  # later stages on the left
        # drop diagonals that cancel to rounding noise (structural zeros)
        out.append({d: D for d, D in G.items() if np.max(np.abs(D)) > 1e-9})
        pos += r
    return out


def coeff_to_slot_factors(n: int, iters: int) -> list:
    """fftIter matrices in diagonal form, in application order, whose product
    is R V^-1 (slots z -> bit-reversed coefficient pairs R w)."""
    return _groups(n, iters, True)


def slot_to_coeff_factors(n: int, iters: int) -> list:
    """fftIter matrices in diagonal form, in application order, whose product
    is V R (slots R w -> z)."""
    return _groups(n, iters, False)


# --------------------------------------------------------------- homomorphic

def rotation_galois(d: int, N: int) -> int:
    """The automorphism rotating the slots right by d (1 for d = 0)."""
    return pow(5, -d, 2 * N) if d % (N // 2) else 1


def diagonal_plaintext(pr, D: np.ndarray, scale: float, level: int) -> np.ndarray:
    """A diagonal encoded at `scale` over Q_level U P, [level + K][N],
    evaluation form (the plaintext format of the hoisted PtMatVecMult)."""
    mods = pr.ext_mods(level)
    return O.ntt(O.lift_signed(encode(D, scale), pr.log_n, mods), pr.log_n, mods)


def linear_layer(pr, ct: np.ndarray, level: int, factors: list, keys: dict):
    """Each factor as one PtMatVecMult (offset d: rotation right by d with
    keys[d]; offset 0: no key) with its diagonals encoded at scale
    q_(level-1), then Rescale.  Returns (ciphertext, level, steps) with
    steps[i] = (level, galois list, key list, plaintext list, output before
    Rescale)."""
    steps = []
    for G in factors:
        ds = sorted(G)
        gals = [rotation_galois(d, pr.n) for d in ds]
        ksks = [keys[d] if d else None for d in ds]
        pts = [diagonal_plaintext(pr, G[d], float(pr.q[level - 1]), level) for d in ds]
        pre = O.ptmatvec(pr, ct, level, gals, ksks, pts)
        steps.append((level, gals, ksks, pts, pre))
        ct = O.rescale(pr, pre, level)
        level -= 1
    return ct, level, steps
