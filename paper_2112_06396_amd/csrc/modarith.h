// Device-side modular arithmetic for 50-bit primes held in 64-bit words
// (Sec. 2.2: conditional-subtraction add, Barrett reduction, lazy sums,
// Shoup constant multiplication).  Built from the 32-bit integer VALU ops of
// gfx950 (v_mad_u64_u32, v_mul_hi_u32, v_mul_lo_u32); no floating point.
//
// Ranges.  Every prime satisfies 2^49 < q < 2^50.  Kernels keep values lazy
// (not fully reduced) inside a computation and reduce to [0, q) before any
// value leaves through the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hks {

typedef unsigned __int128 u128;

// Shoup: x * w mod q for a constant w < q with wp = floor(w * 2^64 / q).
// Any x < 2^64; result in [0, 2q).  (Shoup's method: the quotient estimate
// hi64(x * wp) is low by at most one.)
__device__ __forceinline__ uint64_t mul_shoup_lazy(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
    uint64_t qh = __umul64hi(x, wp);
    return x * w - qh * q;
}

// The same with nq = 2^64 - q: x*w + qh*nq = x*w - qh*q (mod 2^64), so the
// product terms accumulate in carry-free 64-bit multiply-adds instead of a
// subtraction with borrow.
__device__ __forceinline__ uint64_t mul_shoup_lazy_nq(uint64_t x, uint64_t w, uint64_t wp, uint64_t nq) {
    uint64_t qh = __umul64hi(x, wp);
    return x * w + qh * nq;
}

__device__ __forceinline__ uint64_t csub(uint64_t x, uint64_t m) { return x >= m ? x - m : x; }

__device__ __forceinline__ uint64_t mul_shoup(uint64_t x, uint64_t w, uint64_t wp, uint64_t q) {
    return csub(mul_shoup_lazy(x, w, wp, q), q);
}

// Barrett reduction of a 128-bit value X = hi*2^64 + lo < 2^111 for
// 2^49 < q < 2^50, with mu = floor(2^112 / q) (< 2^63).  The estimate
// floor((X >> 48) * mu / 2^64) is at most one below floor(X / q), so the
// remainder lands in [0, 2q) before the last conditional subtraction.
__device__ __forceinline__ uint64_t reduce128(uint64_t hi, uint64_t lo, uint64_t q, uint64_t mu) {
    uint64_t xs = (hi << 16) | (lo >> 48);
    uint64_t qh = __umul64hi(xs, mu);
    uint64_t r = lo - qh * q;
    return csub(r, q);
}

// The same with nq = 2^64 - q: the remainder lo - qh q is formed as
// lo + qh nq (mod 2^64), a carry-free multiply-add.
__device__ __forceinline__ uint64_t reduce128(uint64_t hi, uint64_t lo, uint64_t q, uint64_t mu, uint64_t nq) {
    uint64_t xs = (hi << 16) | (lo >> 48);
    uint64_t qh = __umul64hi(xs, mu);
    return csub(lo + qh * nq, q);
}

__device__ __forceinline__ uint64_t reduce64(uint64_t x, uint64_t q, uint64_t mu, uint64_t nq) {
    return reduce128(0, x, q, mu, nq);
}

// Reduction of any 64-bit x to [0, q) (same Barrett with hi = 0).
__device__ __forceinline__ uint64_t reduce64(uint64_t x, uint64_t q, uint64_t mu) {
    return reduce128(0, x, q, mu);
}

// 128-bit accumulator for lazy sums of products (Sec. 2.2: reduce once at the end).
struct Acc128 {
    uint64_t lo, hi;
    __device__ __forceinline__ Acc128() : lo(0), hi(0) {}
    __device__ __forceinline__ explicit Acc128(uint64_t v) : lo(v), hi(0) {}
    __device__ __forceinline__ void mac(uint64_t a, uint64_t b) {
        u128 p = (u128)a * b;
        uint64_t plo = (uint64_t)p, phi = (uint64_t)(p >> 64);
        lo += plo;
        hi += phi + (lo < plo ? 1 : 0);
    }
    __device__ __forceinline__ uint64_t reduce(uint64_t q, uint64_t mu) const { return reduce128(hi, lo, q, mu); }
};

// Generic x * y mod q for two variables (x * y < 2^111): 128-bit product then Barrett.
__device__ __forceinline__ uint64_t mul_mod(uint64_t x, uint64_t y, uint64_t q, uint64_t mu) {
    u128 p = (u128)x * y;
    return reduce128((uint64_t)(p >> 64), (uint64_t)p, q, mu);
}

__device__ __forceinline__ uint64_t mul_mod(uint64_t x, uint64_t y, uint64_t q, uint64_t mu, uint64_t nq) {
    u128 p = (u128)x * y;
    return reduce128((uint64_t)(p >> 64), (uint64_t)p, q, mu, nq);
}

// Montgomery product x w 2^-64 mod q, in [0, 2q) when x w < q 2^64 (the
// butterflies' lazy x < 4q and w < q with 50-bit q give x w < 2^102): with
// T = x w and m = (T mod 2^64) q' mod 2^64, q' = -q^-1 mod 2^64, T + m q is
// a multiple of 2^64 and (T + m q) / 2^64 = hi(T) + hi(m q) + [lo(T) != 0]
// (the low words sum to 0 or to 2^64), below T / 2^64 + q.
__device__ __forceinline__ uint64_t mont_lazy(uint64_t x, uint64_t w, uint64_t q, uint64_t qinv) {
    const u128 t = (u128)x * w;
    const uint64_t lo = (uint64_t)t, hi = (uint64_t)(t >> 64);
    const uint64_t m = lo * qinv;
    return hi + __umul64hi(m, q) + (lo != 0 ? 1u : 0u);
}

__device__ __forceinline__ uint64_t add_mod(uint64_t x, uint64_t y, uint64_t q) { return csub(x + y, q); }
__device__ __forceinline__ uint64_t sub_mod(uint64_t x, uint64_t y, uint64_t q) { return csub(x + q - y, q); }

}  // namespace hks
