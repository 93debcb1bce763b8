"""Pure-Python big-integer definitions for tiny N (test infrastructure only).

These are the mathematical definitions the C oracle is pinned against; they
share no code with it.  Everything is Python ``int`` arithmetic, so there is
no word-size reasoning to get wrong.

  - NTT by direct evaluation (Sec. 2.3: N evaluations at fixed roots of
    unity), slot j at psi^(2*brv(j)+1);
  - negacyclic schoolbook product in Z_q[X]/(X^N + 1);
  - Chinese remaindering (Sec. 2.2, RNS);
  - the automorphism X -> X^g on integer polynomials;
  - the canonical-embedding slot values m(zeta^(5^j)), zeta = exp(i*pi/N), in
    float64, used only to pin which Galois element realizes the paper's
    rotation phi_k (worked example in Sec. 2.1).
"""
from __future__ import annotations

import cmath
import math


def brv(x: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (x & 1)
        x >>= 1
    return r


def is_prime(n: int) -> bool:
    """trial division (slow; for cross-checking on a few values)"""
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    i = 3
    while i * i <= n:
        if n % i == 0:
            return False
        i += 2
    return True


def ntt_direct(x, q: int, psi: int):
    n = len(x)
    bits = n.bit_length() - 1
    out = []
    for j in range(n):
        e = 2 * brv(j, bits) + 1
        root = pow(psi, e, q)
        acc, pw = 0, 1
        for i in range(n):
            acc += int(x[i]) * pw
            pw = pw * root % q
        out.append(acc % q)
    return out


def ntt_point(x, q: int, psi: int, j: int) -> int:
    """one output of the NTT by direct evaluation"""
    n = len(x)
    bits = n.bit_length() - 1
    root = pow(psi, 2 * brv(j, bits) + 1, q)
    acc, pw = 0, 1
    for i in range(n):
        acc = (acc + int(x[i]) * pw) % q
        pw = pw * root % q
    return acc


def negacyclic_mul(a, b, q: int):
    n = len(a)
    out = [0] * n
    for i in range(n):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                out[k] += ai * int(b[j])
            else:
                out[k - n] -= ai * int(b[j])
    return [v % q for v in out]


def crt(residues, moduli) -> int:
    M = 1
    for m in moduli:
        M *= int(m)
    x = 0
    for r, m in zip(residues, moduli):
        m = int(m)
        Mi = M // m
        x += int(r) * Mi * pow(Mi % m, -1, m)
    return x % M


def prod(vals) -> int:
    r = 1
    for v in vals:
        r *= int(v)
    return r


def automorph_int(a, g: int):
    """integer polynomial a(X) -> a(X^g) mod X^N + 1"""
    n = len(a)
    out = [0] * n
    for i in range(n):
        e = (i * g) % (2 * n)
        if e < n:
            out[e] += int(a[i])
        else:
            out[e - n] -= int(a[i])
    return out


def slots(m, n_slots: int | None = None):
    """m(zeta^(5^j)) for j < N/2, zeta = exp(i pi / N) (float64 complex)"""
    n = len(m)
    ns = n // 2 if n_slots is None else n_slots
    out = []
    for j in range(ns):
        e = pow(5, j, 2 * n)
        z = cmath.exp(1j * math.pi * e / n)
        acc = 0j
        zp = 1 + 0j
        for i in range(n):
            acc += int(m[i]) * zp
            zp *= z
        out.append(acc)
    return out
