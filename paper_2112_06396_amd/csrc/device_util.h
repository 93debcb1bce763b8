// Small device helpers shared by the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

namespace hks {

__device__ __forceinline__ uint32_t brev_n(uint32_t x, uint32_t n) { return __brev(x) >> (32 - n); }

// Source slot of output slot j under X -> X^g in the bit-reversed evaluation
// order: slot j holds a(psi^(2 brv(j) + 1)); psi^((2 brv(j)+1) g) is held by
// slot brv(((2 brv(j) + 1) g mod 2N - 1) / 2).  Aligned blocks of 2^b slots
// map onto aligned blocks of 2^b slots (the low bits of brv(j) map among
// themselves), so a gather over a tile reads one whole tile.
__device__ __forceinline__ uint32_t aut_eval_src(uint32_t j, uint32_t g, uint32_t n) {
    uint32_t k = brev_n(j, n);
    uint32_t odd = ((2u * k + 1u) * g) & ((2u << n) - 1u);
    return brev_n((odd - 1u) >> 1, n);
}

// 128-bit sum of products of residues, kept as three 64-bit words
// (lo + mid * 2^32 + hi * 2^64) so that each product costs three
// v_mad_u64_u32: x = xh 2^32 + xl, k = kh 2^32 + kl with xh < 2^24,
// kh < 2^18 (x < 2^56, k < 2^50).
struct MacAcc {
    uint64_t lo, mid, hi;
    __device__ __forceinline__ MacAcc() : lo(0), mid(0), hi(0) {}
    __device__ __forceinline__ void mac(uint64_t x, uint64_t k) {
        const uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32);
        const uint32_t kl = (uint32_t)k, kh = (uint32_t)(k >> 32);
        const uint64_t p0 = (uint64_t)xl * kl;
        const uint64_t t = lo + p0;
        hi += (t < lo) ? 1u : 0u;
        lo = t;
        mid += (uint64_t)xl * kh;
        mid += (uint64_t)xh * kl;
        hi += (uint64_t)xh * kh;
    }
    // reduce the (< 2^111) sum modulo q (Barrett, mu = floor(2^112 / q))
    __device__ __forceinline__ uint64_t reduce(uint64_t q, uint64_t mu) const {
        const uint64_t l = lo + (mid << 32);
        const uint64_t h = hi + (mid >> 32) + ((l < lo) ? 1u : 0u);
        return reduce128(h, l, q, mu);
    }
};

// Sum of products y_i * k_i of canonical 50-bit residues with y and k split
// into 25-bit halves: each product adds y0 k0, y0 k1 + y1 k0 and y1 k1 to
// three 64-bit sums (one v_mad_u64_u32 each, no carries for up to 16 terms:
// every partial product is < 2^50).  k comes pre-split as k0 | (k1 << 32).
struct Mac25 {
    uint64_t a0, a1, a2;
    __device__ __forceinline__ Mac25() : a0(0), a1(0), a2(0) {}
    __device__ __forceinline__ void mac(uint32_t y0, uint32_t y1, uint64_t ksplit) {
        const uint32_t k0 = (uint32_t)ksplit, k1 = (uint32_t)(ksplit >> 32);
        a0 += (uint64_t)y0 * k0;
        a1 += (uint64_t)y0 * k1;
        a1 += (uint64_t)y1 * k0;
        a2 += (uint64_t)y1 * k1;
    }
    // a0 + a1 2^25 + a2 2^50 (< 2^105) reduced modulo q (mu = floor(2^112 / q),
    // nq = 2^64 - q)
    __device__ __forceinline__ uint64_t reduce(uint64_t q, uint64_t mu, uint64_t nq) const {
        const uint64_t l1 = a1 << 25, l2 = a2 << 50;
        uint64_t lo = a0 + l1;
        uint64_t hi = (a1 >> 39) + (a2 >> 14) + ((lo < l1) ? 1u : 0u);
        const uint64_t lo2 = lo + l2;
        hi += (lo2 < l2) ? 1u : 0u;
        return reduce128(hi, lo2, q, mu, nq);
    }
};

// Counter-based generator Philox4x32-10 (Salmon et al., SC 2011): ten
// rounds, each multiplying words 0 and 2 by the round constants and mixing
// the products' halves with words 1 and 3 and the round key; the key grows
// by the Weyl increments between rounds.  Returns words 0..2 of the output.
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                              uint32_t k1, uint32_t &o0, uint32_t &o1, uint32_t &o2) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0;
    o1 = c1;
    o2 = c2;
}

// Entry (digit j, key limb kappa, slot i) of a seeded key's uniform rows:
// the generator's low 96 bits for counter (i, kappa, j, 0x4B53) and key
// (seed mod 2^32, seed >> 32), reduced mod the limb's prime (Barrett on a
// value below 2^96).
__device__ __forceinline__ uint64_t seeded_key_a(uint64_t seed, uint32_t j, uint32_t kappa, uint32_t i, uint64_t q,
                                                 uint64_t mu, uint64_t nq) {
    uint32_t o0, o1, o2;
    philox4x32_10(i, kappa, j, 0x4B53u, (uint32_t)seed, (uint32_t)(seed >> 32), o0, o1, o2);
    return reduce128(o2, ((uint64_t)o1 << 32) | o0, q, mu, nq);
}

__device__ __forceinline__ void split25(uint64_t y, uint32_t &y0, uint32_t &y1) {
    y0 = (uint32_t)y & 0x1FFFFFFu;
    y1 = (uint32_t)(y >> 25);
}

}  // namespace hks
