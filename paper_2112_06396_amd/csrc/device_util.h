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

}  // namespace hks
