"""Pins of the oracle's encoding and factored DFT (bootstrapping's linear
layers, Sec. 3) against the definitions: the canonical embedding evaluated
point by point, the closed-form matrix V[j, k] = zeta^(5^j k), the rotation
direction of the slots, and exact identities of the hoisted PtMatVecMult.
"""
import numpy as np
import pytest

from oracle import bigint as B
from oracle import encoding as C
from oracle import oracle as O
from paper_2112_06396_amd import synth


def _z(g, n):
    return g.uniform(-1, 1, n) + 1j * g.uniform(-1, 1, n)


def test_decode_is_evaluation_at_the_rotation_group():
    """decode(m) equals m(zeta^(5^j)) evaluated term by term (N = 16, 32)."""
    for log_n in (4, 5):
        n = 1 << log_n
        m = synth.small_uniform(synth.rng(30 + log_n), n, 1000)
        ref = np.array(B.slots(list(m)))
        assert np.max(np.abs(C.decode(m, 1.0) - ref)) < 1e-9 * n * 1000


def test_vandermonde_is_unitary_up_to_n():
    for n in (4, 16, 64):
        V = C.vandermonde(n)
        assert np.max(np.abs(V.conj().T @ V - n * np.eye(n))) < 1e-9


def test_encode_inverts_decode():
    """decode(encode(z)) = z up to the rounding of N coefficients (each
    rounding moves every slot by at most 1/(2 Delta))."""
    n = 512
    g = synth.rng(40)
    z = _z(g, n)
    for scale in (2.0 ** 20, 2.0 ** 40):
        m = C.encode(z, scale)
        assert m.shape == (2 * n,)
        assert np.max(np.abs(C.decode(m, scale) - z)) <= n / scale
    # and encode(decode(m)) = m for integer m (the map is a bijection)
    m = synth.small_uniform(g, 2 * n, 1 << 20)
    assert np.array_equal(C.encode(C.decode(m, 1.0), 1.0), m)


def test_slot_rotation_is_the_automorphism():
    """Rotating the slots right by d (entry j <- j - d, the paper's phi_d) is
    X -> X^(5^-d mod 2N) on the plaintext, the convention every diagonal
    offset below relies on."""
    N = 64
    n = N // 2
    g = synth.rng(41)
    m = synth.small_uniform(g, N, 1000)
    z = C.decode(m, 1.0)
    for d in (1, 3, n - 1, 7):
        md = B.automorph_int(list(m), pow(5, -d, 2 * N))
        assert np.max(np.abs(C.decode(md, 1.0) - np.roll(z, d))) < 1e-8


@pytest.mark.parametrize("n", [2, 8, 32, 256])
def test_factors_multiply_to_the_dft(n):
    """SlotToCoeff's factors multiply to V R and CoeffToSlot's to R V^-1,
    with V from its closed form and R the bit reversal; grouping only
    multiplies stages out (a group of r stages has at most 2^(r+1) - 1
    diagonals, and exactly that many when no offsets wrap)."""
    V = C.vandermonde(n)
    R = np.eye(n)[C.bit_reverse_perm(n)]
    logn = n.bit_length() - 1
    for iters in sorted({1, min(3, logn), logn}):
        st, ct = C.slot_to_coeff_factors(n, iters), C.coeff_to_slot_factors(n, iters)
        assert len(st) == len(ct) == iters
        M = np.eye(n)
        for G in st:
            M = C.to_dense(G, n) @ M
        assert np.max(np.abs(M - V @ R)) < 1e-10 * n
        Mi = np.eye(n)
        for G in ct:
            Mi = C.to_dense(G, n) @ Mi
        assert np.max(np.abs(Mi @ V - R)) < 1e-10 * n
        # diagonal counts (SlotToCoeff groups cover S_2.. upward: offsets 2^s)
        pos = 0
        for r, G in zip(C.radices(logn, iters), st):
            top = 1 << (pos + r - 1)  # largest half-size in the group
            wraps = 2 * (2 * top - 1) >= n
            assert len(G) <= 2 ** (r + 1) - 1
            if not wraps:
                assert len(G) == 2 ** (r + 1) - 1
            pos += r


def test_radices_follow_the_paper_example():
    """n = 2^16 with three iterations: radices 2^5, 2^5, 2^6; with five:
    four of 2^3 and one of 2^4 (Sec. 3)."""
    assert C.radices(16, 3) == [5, 5, 6]
    assert C.radices(16, 5) == [3, 3, 3, 3, 4]


def test_ptmatvec_zero_rotation_term_is_an_exact_ptmult():
    """A PtMatVecMult whose only diagonal has offset 0 (no key) is PModUp of
    the input times M, then one ModDown, which is exact on multiples of P:
    the result equals PtMult bit for bit."""
    pr = O.make_params(10, 5, 2, 3)
    g = synth.rng(42)
    level = 5
    ct = np.stack([synth.uniform_residues(g, pr.q[:level], pr.n) for _ in range(2)])
    pt = synth.uniform_residues(g, pr.ext_mods(level), pr.n)
    out = O.ptmatvec(pr, ct, level, [1], [None], [pt])
    assert np.array_equal(out, O.ptmult(pr, ct, pt[:level], level, False))


def _crt_centered(res, mods):
    Q = B.prod(mods)
    vals = [B.crt([int(res[i][c]) for i in range(len(mods))], mods) for c in range(res.shape[1])]
    return [v - Q if v > Q // 2 else v for v in vals]


def _keys(pr, s, g, factors, keys):
    for G in factors:
        for d in G:
            if d and d not in keys:
                keys[d] = O.rotation_key(pr, s, C.rotation_galois(d, pr.n), g)
    return keys


def test_coeff_to_slot_and_back_through_the_oracle():
    """CoeffToSlot at N = 2^10 (n = 512 slots, three PtMatVecMult of 8, 15
    and 15 diagonals, each followed by Rescale) decrypts and decodes to R w,
    the bit-reversed coefficient pairs of the input; SlotToCoeff (15, 15, 8
    diagonals, the same rotation indices) then returns the slots z."""
    pr = O.make_params(10, 8, 3, 3)
    g = synth.rng(43)
    s = synth.ternary(g, pr.n)
    n = pr.n // 2
    z = _z(g, n)
    scale = 2.0 ** 40
    ct = O.encrypt(pr, s, C.encode(z, scale), pr.L, g)
    factors = C.coeff_to_slot_factors(n, 3)
    assert [len(G) for G in factors] == [8, 15, 15]
    keys = _keys(pr, s, g, factors, {})
    mid, level, _ = C.linear_layer(pr, ct, pr.L, factors, keys)
    assert level == pr.L - 3
    m = _crt_centered(O.decrypt_coef(pr, s, mid, level), [int(q) for q in pr.q[:level]])
    want = C.encode_w(z)[C.bit_reverse_perm(n)]
    assert np.max(np.abs(C.decode(m, scale) - want)) < 1e-6
    n_keys = len(keys)
    back_f = C.slot_to_coeff_factors(n, 3)
    assert [len(G) for G in back_f] == [15, 15, 8]
    _keys(pr, s, g, back_f, keys)
    back, level, _ = C.linear_layer(pr, mid, level, back_f, keys)
    assert len(keys) == n_keys  # same rotation indices as CoeffToSlot
    m = _crt_centered(O.decrypt_coef(pr, s, back, level), [int(q) for q in pr.q[:level]])
    assert np.max(np.abs(C.decode(m, scale) - z)) < 1e-5
