// Negacyclic NTT / iNTT passes for gfx950 (Sec. 2.3): the device-side
// building blocks shared by the pass kernels and the kernels that fuse
// key-switching steps into them (ksk.hip).
//
// Structure.  N = 2^n is viewed as a 2^n1 x 2^n2 matrix (row r, column c,
// element j = r*2^n2 + c).  The forward transform is the merged Cooley-Tukey
// negacyclic NTT with bit-reversed output: stage s (s = 0..n-1) pairs j and
// j + N/2^(s+1) with twiddle psi^brv(2^s + (j >> (n-s))).  Stages 0..n1-1 only
// combine elements of one column (the "column pass"), stages n1..n-1 only
// elements of one row (the "row pass").  The inverse runs Gentleman-Sande
// butterflies in reverse order (row pass first) with N^-1 and any per-limb
// scale folded into the last stage.
//
// A pass kernel loads a tile of LINES lines into LDS with coalesced accesses
// (16 columns = 128-byte segments for the column pass, whole rows for the row
// pass), runs phases of up to four stages with 16 elements per thread in
// registers (each distinct twiddle loaded once per stage), exchanging through
// LDS between phases, and stores coalesced.  Values are lazy between stages:
// forward values grow by < 2q per stage (< 35q < 2^56 after 16 stages),
// inverse values stay in [0, 2q).
//
// Fusions (cache-oriented ideas of the paper, Sec. 4, recast for LDS):
//   ksk_rows  KSKInnerProd streamed per target limb and row tile; for the
//             special-prime limbs it goes on with the inverse row pass of
//             ModDown on chip (P limbs first);
//   IO_MDEPI  row pass of the ModDown correction followed by
//             (u - z) * P^-1 (+ the automorphed b of Rotate).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "hks_internal.h"
#include "modarith.h"

namespace hks {

template <int LOGS, int LINES, bool COLS, int E = 16>
struct Tile {
    static constexpr int S = 1 << LOGS;
    static constexpr int T = S / E;          // threads per line
    static constexpr int NT = LINES * T;     // threads per block
    static constexpr int EPT = E;            // elements per thread
    static constexpr int ROWP = S + S / 16;  // padded row length (row tiles)
    static constexpr int COLP = LINES + 1;   // padded k-row length (column tiles)
    static constexpr int WORDS = COLS ? S * COLP : LINES * ROWP;
    __device__ static __forceinline__ int idx(int line, int k) {
        return COLS ? k * COLP + line : line * ROWP + k + (k >> 4);
    }
};

// Phases of a pass over the LOGS bits of the sub-index k with R = log2 of
// the elements per thread: P0 = [LOGS-R, LOGS), P1 = [max(LOGS-2R, 0),
// LOGS-R), P2 = [0, LOGS-2R) when LOGS > 2R.  The forward pass runs P0, P1,
// P2 (high bits first); the inverse runs them in reverse.
template <int LOGS, int R = 4>
struct Phases {
    static_assert(LOGS > R && LOGS <= 3 * R, "a pass has two or three phases");
    static constexpr int P0L = LOGS - R, P0H = LOGS;
    static constexpr int P1L = (LOGS - 2 * R) > 0 ? (LOGS - 2 * R) : 0, P1H = LOGS - R;
    static constexpr int P2L = 0, P2H = (LOGS - 2 * R) > 0 ? (LOGS - 2 * R) : 0;
    static constexpr bool THREE = LOGS > 2 * R;
};

template <int E>
struct Log2 {
    static constexpr int value = E == 8 ? 3 : 4;
    static_assert(E == 8 || E == 16, "8 or 16 elements per thread");
};

// Element e (0..E-1) of thread t in the layout of phase [LO, HI): the
// thread holds every value of bits [LO, HI) of k for E >> (HI-LO) values of
// the other bits.  [LOGS-R, LOGS) gives k = e*T + t (consecutive threads on
// consecutive k); [0, b) gives k = E t + e (each thread a contiguous run).
template <int LO, int HI, int E = 16>
__device__ __forceinline__ int k_of(int t, int e) {
    constexpr int B = HI - LO, G = E >> B;
    const int v = e & ((1 << B) - 1), g = e >> B;
    const int r = t * G + g;
    return ((r >> LO) << HI) | (v << LO) | (r & ((1 << LO) - 1));
}

#ifndef HKS_TW_HOIST
#define HKS_TW_HOIST 1
#endif
constexpr bool TW_HOIST = HKS_TW_HOIST != 0;  // pass kernels load a phase's twiddles up front
// Row passes load all their twiddles before the first butterfly (measured:
// Rotate -1.4%); column passes, whose few twiddles are cache hits, per phase
// (loading all up front measured no better).
constexpr bool TW_PRE_ROWS = true;
constexpr bool TW_PRE_COLS = false;

// Twiddle sources.  The butterfly group m = k >> (bit+1) of local stage ls
// (0-based within the pass) uses
//   column pass: table index 2^ls + m;
//   row pass:    table index ((2^n1 + r) << ls) + m for row r.
// Elements whose k agree above `bit` share the twiddle.
struct TwCols {
    const Shoup *tw;
    __device__ __forceinline__ Shoup operator()(int ls, uint32_t m) const { return tw[(1u << ls) + m]; }
};
struct TwRows {
    const Shoup *tw;
    uint32_t row, n1;
    __device__ __forceinline__ Shoup operator()(int ls, uint32_t m) const {
        return tw[(((1u << n1) + row) << ls) + m];
    }
};
// Row twiddles in Montgomery form (w 2^64 mod q): the butterfly multiplies
// with a Montgomery product, from 8 bytes per twiddle where a Shoup pair
// takes 16.
struct TwRowsM {
    const uint64_t *tw;  // the modulus's [N] table
    uint32_t row, n1;
    __device__ __forceinline__ uint64_t operator()(int ls, uint32_t m) const {
        return tw[(((1u << n1) + row) << ls) + m];
    }
};

// Row passes of 8 or more stages (N >= 2^15 at the default split) read
// their twiddles in Montgomery form: half the table bytes for one more
// multiply-high on the butterfly's path.  Shorter passes belong to small
// rings, whose launches are a few blocks each and bound by the latency of
// that path (measured at N = 2^12: Rotate 41.6 us with Shoup pairs, 46.9 us
// with Montgomery twiddles), so they keep Shoup pairs.
template <int LOGS>
constexpr bool MONT_ROWS = LOGS >= 8;

// The butterfly's product with a twiddle: Shoup with a (w, w') pair, or
// Montgomery with a Montgomery-form twiddle.
__device__ __forceinline__ uint64_t tw_mul(uint64_t x, const Shoup &w, uint64_t, uint64_t nq, uint64_t) {
    return mul_shoup_lazy_nq(x, w.w, w.wp, nq);
}
__device__ __forceinline__ uint64_t tw_mul(uint64_t x, uint64_t wm, uint64_t q, uint64_t, uint64_t qinv) {
    return mont_lazy(x, wm, q, qinv);
}

// The row twiddles of `lines` consecutive rows from row0, staged in LDS: for
// local stage ls the rows' entries ((2^n1 + r) << ls) + m form one
// contiguous run of lines << ls entries, stored at lines (2^ls - 1).
template <int LINES>
struct TwRowsLds {
    const Shoup *tw;  // LDS
    uint32_t line;    // row - row0
    __device__ __forceinline__ Shoup operator()(int ls, uint32_t m) const {
        return tw[LINES * ((1u << ls) - 1) + (line << ls) + m];
    }
};
template <int LOGS, int LINES>
__device__ __forceinline__ void stage_row_twiddles(Shoup *lds_tw, const Shoup *__restrict__ tw, uint32_t row0,
                                                   uint32_t n1) {
#pragma unroll
    for (int ls = 0; ls < LOGS; ++ls) {
        const Shoup *src = tw + (((1u << n1) + row0) << ls);
        Shoup *dst = lds_tw + LINES * ((1u << ls) - 1);
        for (uint32_t i = threadIdx.x; i < (LINES << ls); i += blockDim.x) dst[i] = src[i];
    }
}
// Order of LDS accesses within a wave: a wave's LDS operations take effect
// in issue order, so only the compiler must not move them across
// (wavefront-scope fences around a wave barrier; no instruction is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// The synchronization of a pass's LDS exchanges.  A column's threads span
// the block (line = tid % LINES): block barrier.  A row's T threads are
// consecutive and T divides 64 (line = tid / T), so each row lives in one
// wave and its exchanges only need wave_sync; the block's waves then run
// their passes independently (measured against block barriers: Rotate
// -2.5%, the key-switch kernel -7%).
template <bool COLS>
__device__ __forceinline__ void pass_sync() {
    if constexpr (COLS) __syncthreads();
    else wave_sync();
}

// The twiddles of one phase (layout [LO, HI)) for the thread: E >> (vb+1)
// distinct ones per stage (none for the folded last inverse stage).
template <int LOGS, bool FWD, bool FOLD, int LO, int HI, int E, typename TW, typename TV>
__device__ __forceinline__ void phase_tw(TV (&w)[HI - LO][E / 2], int t, const TW &tws) {
    constexpr int B = HI - LO, H = E / 2;
#pragma unroll
    for (int st = 0; st < B; ++st) {
        const int bit = FWD ? (HI - 1 - st) : (LO + st);
        const int vb = bit - LO;
        const int ls = LOGS - 1 - bit;
#pragma unroll
        for (int key = 0; key < H; ++key) {
            if (key < (E >> (vb + 1)) && !(FOLD && ls == 0)) {
                const uint32_t k = (uint32_t)k_of<LO, HI, E>(t, key << (vb + 1));
                w[st][key] = tws(ls, k >> (bit + 1));
            }
        }
    }
}

// The butterflies of one phase with its twiddles already in registers.
template <int LOGS, bool FWD, bool FOLD, int LO, int HI, int E, typename TV>
__device__ __forceinline__ void phase_bfly(uint64_t (&x)[E], uint64_t q, uint64_t nq, uint64_t qinv,
                                           const TV (&w)[HI - LO][E / 2], const LastInv &fold) {
    constexpr int B = HI - LO, H = E / 2;
    const uint64_t q2 = 2 * q;
#pragma unroll
    for (int st = 0; st < B; ++st) {
        const int bit = FWD ? (HI - 1 - st) : (LO + st);
        const int vb = bit - LO;
        const bool fold_stage = FOLD && (LOGS - 1 - bit) == 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if ((e >> vb) & 1) continue;
            const int e2 = e + (1 << vb);
            const TV wc = w[st][(e >> (vb + 1)) & (H - 1)];
            if (FWD) {
                const uint64_t u = x[e];
                const uint64_t tv = tw_mul(x[e2], wc, q, nq, qinv);
                x[e] = u + tv;
                x[e2] = u + q2 - tv;
            } else {
                const uint64_t u = x[e], v = x[e2];
                if (fold_stage) {
                    x[e] = mul_shoup(u + v, fold.c.w, fold.c.wp, q);
                    x[e2] = mul_shoup(u + q2 - v, fold.cw.w, fold.cw.wp, q);
                } else {
                    x[e] = csub(u + v, q2);
                    x[e2] = tw_mul(u + q2 - v, wc, q, nq, qinv);
                }
            }
        }
    }
}

// The butterflies of one phase on the thread's E registers (layout [LO, HI)).
// Each stage loads E >> (vb+1) distinct twiddles.  With FOLD (the inverse
// column pass) the global last inverse stage multiplies by the folded
// constants instead.
template <int LOGS, bool FWD, bool FOLD, int LO, int HI, bool HOIST, int E, typename TW>
__device__ __forceinline__ void phase_regs(uint64_t (&x)[E], int t, uint64_t q, uint64_t nq, const TW &tws,
                                           const LastInv &fold, uint64_t qinv) {
    constexpr int B = HI - LO, H = E / 2;
    using TV = decltype(tws(0, 0u));
    const uint64_t q2 = 2 * q;
    // HOIST: every twiddle of the phase loaded up front (E >> (vb+1) per
    // stage), one memory latency per phase instead of one per stage, for
    // more registers
    TV wall[HOIST ? B : 1][H];
#pragma unroll
    for (int st = 0; st < (HOIST ? B : 0); ++st) {
        const int bit = FWD ? (HI - 1 - st) : (LO + st);
        const int vb = bit - LO;
        const int ls = LOGS - 1 - bit;
#pragma unroll
        for (int key = 0; key < H; ++key) {
            if (key < (E >> (vb + 1)) && !(FOLD && ls == 0)) {
                const uint32_t k = (uint32_t)k_of<LO, HI, E>(t, key << (vb + 1));
                wall[st][key] = tws(ls, k >> (bit + 1));
            }
        }
    }
#pragma unroll
    for (int st = 0; st < B; ++st) {
        const int bit = FWD ? (HI - 1 - st) : (LO + st);
        const int vb = bit - LO;
        const int ls = LOGS - 1 - bit;  // stage within this pass
        const bool fold_stage = FOLD && ls == 0;
        TV wc[H];
#pragma unroll
        for (int key = 0; key < H; ++key) {
            if (HOIST) {
                wc[key] = wall[HOIST ? st : 0][key];
            } else if (key < (E >> (vb + 1)) && !fold_stage) {
                const uint32_t k = (uint32_t)k_of<LO, HI, E>(t, key << (vb + 1));
                wc[key] = tws(ls, k >> (bit + 1));
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if ((e >> vb) & 1) continue;
            const int e2 = e + (1 << vb);
            const TV w = wc[(e >> (vb + 1)) & (H - 1)];
            if (FWD) {
                const uint64_t u = x[e];
                const uint64_t tv = tw_mul(x[e2], w, q, nq, qinv);
                x[e] = u + tv;
                x[e2] = u + q2 - tv;
            } else {
                const uint64_t u = x[e], v = x[e2];
                if (fold_stage) {
                    x[e] = mul_shoup(u + v, fold.c.w, fold.c.wp, q);
                    x[e2] = mul_shoup(u + q2 - v, fold.cw.w, fold.cw.wp, q);
                } else {
                    x[e] = csub(u + v, q2);
                    x[e2] = tw_mul(u + q2 - v, w, q, nq, qinv);
                }
            }
        }
    }
}

template <int LOGS, int LINES, bool COLS, int LO, int HI, int E>
__device__ __forceinline__ void lds_put(uint64_t *lds, const uint64_t (&x)[E], int line, int t) {
    using TL = Tile<LOGS, LINES, COLS, E>;
#pragma unroll
    for (int e = 0; e < E; ++e) lds[TL::idx(line, k_of<LO, HI, E>(t, e))] = x[e];
}

template <int LOGS, int LINES, bool COLS, int LO, int HI, int E>
__device__ __forceinline__ void lds_get(const uint64_t *lds, uint64_t (&x)[E], int line, int t) {
    using TL = Tile<LOGS, LINES, COLS, E>;
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = lds[TL::idx(line, k_of<LO, HI, E>(t, e))];
}

// A whole pass on registers.  On entry x is in the first phase's layout
// (forward: P0, inverse: P2 or P1), on exit in the last one's (forward: P1 or
// P2, inverse: P0).  The LDS tile carries the exchanges between phases; the
// caller synchronizes before this tile is written again.  Work is done only
// where `active` holds, but every thread reaches every barrier.
// With PRE every twiddle of the pass is loaded before the first butterfly:
// one memory latency for the pass (overlapping the data loads the caller
// issued before) instead of one per phase, for their registers.
template <int LOGS, int LINES, bool COLS, bool FWD, bool HOIST, int E = 16, bool PRE = false, typename TW>
__device__ __forceinline__ void pass_regs(bool active, uint64_t (&x)[E], uint64_t *lds, int line, int t, uint64_t q,
                                          uint64_t nq, const TW &tws, const LastInv &fold, uint64_t qinv = 0) {
    using P = Phases<LOGS, Log2<E>::value>;
    using TV = decltype(tws(0, 0u));
    constexpr bool FOLD = !FWD && COLS;
    static_assert(COLS || 64 % Tile<LOGS, LINES, COLS, E>::T == 0, "a row's threads are in one wave");
    if constexpr (PRE) {
        constexpr int H = E / 2;
        TV w0[P::P0H - P::P0L][H], w1[P::P1H - P::P1L][H], w2[P::THREE ? P::P2H - P::P2L : 1][H];
        phase_tw<LOGS, FWD, FOLD, P::P0L, P::P0H, E>(w0, t, tws);
        phase_tw<LOGS, FWD, FOLD, P::P1L, P::P1H, E>(w1, t, tws);
        if constexpr (P::THREE) phase_tw<LOGS, FWD, FOLD, P::P2L, P::P2H, E>(w2, t, tws);
        if (FWD) {
            if (active) {
                phase_bfly<LOGS, true, FOLD, P::P0L, P::P0H, E>(x, q, nq, qinv, w0, fold);
                lds_put<LOGS, LINES, COLS, P::P0L, P::P0H, E>(lds, x, line, t);
            }
            pass_sync<COLS>();
            if (active) {
                lds_get<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
                phase_bfly<LOGS, true, FOLD, P::P1L, P::P1H, E>(x, q, nq, qinv, w1, fold);
            }
            if constexpr (P::THREE) {
                pass_sync<COLS>();
                if (active) lds_put<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
                pass_sync<COLS>();
                if (active) {
                    lds_get<LOGS, LINES, COLS, P::P2L, P::P2H, E>(lds, x, line, t);
                    phase_bfly<LOGS, true, FOLD, P::P2L, P::P2H, E>(x, q, nq, qinv, w2, fold);
                }
            }
        } else {
            if constexpr (P::THREE) {
                if (active) {
                    phase_bfly<LOGS, false, FOLD, P::P2L, P::P2H, E>(x, q, nq, qinv, w2, fold);
                    lds_put<LOGS, LINES, COLS, P::P2L, P::P2H, E>(lds, x, line, t);
                }
                pass_sync<COLS>();
                if (active) lds_get<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
                pass_sync<COLS>();
            }
            if (active) {
                phase_bfly<LOGS, false, FOLD, P::P1L, P::P1H, E>(x, q, nq, qinv, w1, fold);
                lds_put<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            }
            pass_sync<COLS>();
            if (active) {
                lds_get<LOGS, LINES, COLS, P::P0L, P::P0H, E>(lds, x, line, t);
                phase_bfly<LOGS, false, FOLD, P::P0L, P::P0H, E>(x, q, nq, qinv, w0, fold);
            }
        }
        return;
    }
    if (FWD) {
        if (active) {
            phase_regs<LOGS, true, FOLD, P::P0L, P::P0H, HOIST, E>(x, t, q, nq, tws, fold, qinv);
            lds_put<LOGS, LINES, COLS, P::P0L, P::P0H, E>(lds, x, line, t);
        }
        pass_sync<COLS>();
        if (active) {
            lds_get<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            phase_regs<LOGS, true, FOLD, P::P1L, P::P1H, HOIST, E>(x, t, q, nq, tws, fold, qinv);
        }
        if constexpr (P::THREE) {
            pass_sync<COLS>();
            if (active) lds_put<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            pass_sync<COLS>();
            if (active) {
                lds_get<LOGS, LINES, COLS, P::P2L, P::P2H, E>(lds, x, line, t);
                phase_regs<LOGS, true, FOLD, P::P2L, P::P2H, HOIST, E>(x, t, q, nq, tws, fold, qinv);
            }
        }
    } else {
        if constexpr (P::THREE) {
            if (active) {
                phase_regs<LOGS, false, FOLD, P::P2L, P::P2H, HOIST, E>(x, t, q, nq, tws, fold, qinv);
                lds_put<LOGS, LINES, COLS, P::P2L, P::P2H, E>(lds, x, line, t);
            }
            pass_sync<COLS>();
            if (active) lds_get<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            pass_sync<COLS>();
        }
        if (active) {
            phase_regs<LOGS, false, FOLD, P::P1L, P::P1H, HOIST, E>(x, t, q, nq, tws, fold, qinv);
            lds_put<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
        }
        pass_sync<COLS>();
        if (active) {
            lds_get<LOGS, LINES, COLS, P::P0L, P::P0H, E>(lds, x, line, t);
            phase_regs<LOGS, false, FOLD, P::P0L, P::P0H, HOIST, E>(x, t, q, nq, tws, fold, qinv);
        }
    }
}

// first / last phase layouts of a pass
template <int LOGS, bool FWD, int E = 16>
struct IoLayout {
    using P = Phases<LOGS, Log2<E>::value>;
    static constexpr int IN_LO = FWD ? P::P0L : (P::THREE ? P::P2L : P::P1L);
    static constexpr int IN_HI = FWD ? P::P0H : (P::THREE ? P::P2H : P::P1H);
    static constexpr int OUT_LO = FWD ? (P::THREE ? P::P2L : P::P1L) : P::P0L;
    static constexpr int OUT_HI = FWD ? (P::THREE ? P::P2H : P::P1H) : P::P0H;
};

// global index of sub-index k of line `lg` (a column, or a row)
template <bool COLS>
__device__ __forceinline__ uint32_t jdx(uint32_t lg, int k, uint32_t n2) {
    return COLS ? (((uint32_t)k << n2) + lg) : ((lg << n2) + (uint32_t)k);
}

// Load / store the thread's E elements of line `lg` in layout [LO, HI).  A
// row pass in a [0, b) layout owns E consecutive words: 16-byte accesses.
template <int LOGS, bool COLS, int LO, int HI, int E = 16>
__device__ __forceinline__ void gload(uint64_t (&x)[E], const uint64_t *__restrict__ src, int t, uint32_t lg,
                                      uint32_t n2) {
    if (!COLS && LO == 0) {
        const ulonglong2 *p = reinterpret_cast<const ulonglong2 *>(src + (lg << n2) + E * t);
#pragma unroll
        for (int i = 0; i < E / 2; ++i) {
            const ulonglong2 v = p[i];
            x[2 * i] = v.x;
            x[2 * i + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = src[jdx<COLS>(lg, k_of<LO, HI, E>(t, e), n2)];
    }
}

template <int LOGS, bool COLS, int LO, int HI, int E = 16>
__device__ __forceinline__ void gstore(const uint64_t (&x)[E], uint64_t *__restrict__ dst, int t, uint32_t lg,
                                       uint32_t n2) {
    if (!COLS && LO == 0) {
        ulonglong2 *p = reinterpret_cast<ulonglong2 *>(dst + (lg << n2) + E * t);
#pragma unroll
        for (int i = 0; i < E / 2; ++i) p[i] = make_ulonglong2(x[2 * i], x[2 * i + 1]);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) dst[jdx<COLS>(lg, k_of<LO, HI, E>(t, e), n2)] = x[e];
    }
}

// thread -> (line, t): column tiles put lines fastest (coalesced columns),
// row tiles put the threads of one line together.
template <int LOGS, int LINES, bool COLS, int E = 16>
__device__ __forceinline__ void thread_coords(int tid, int &line, int &t) {
    using TL = Tile<LOGS, LINES, COLS, E>;
    if (COLS) {
        line = tid % LINES;
        t = tid / LINES;
    } else {
        t = tid % TL::T;
        line = tid / TL::T;
    }
}

// A row pass's input under X -> X^g (bit-reversed evaluation order): the
// aligned block of 2^n2 slots of row lg is the image of one whole source row
// (the automorphism maps aligned blocks onto aligned blocks), so the line's
// threads load that row with contiguous loads (E words each) into the line's
// part of the LDS tile and take their elements from there in the pass's
// input layout (coalesced loads instead of one scattered word per element;
// measured: Rotate -1 us).  A line's threads are one wave's (T
// divides 64), and a wave's LDS operations take effect in order: no block
// barrier.  The caller has synchronized since the tile was last read.
template <int LOGS, int LINES, bool FWD, int E>
__device__ __forceinline__ void gather_row(uint64_t (&x)[E], const uint64_t *src, uint64_t *lds, int line, int t,
                                           uint32_t lg, uint32_t g, uint32_t n, uint32_t n2) {
    using TL = Tile<LOGS, LINES, false, E>;
    using IOL = IoLayout<LOGS, FWD, E>;
    static_assert(TL::T <= 64 && 64 % TL::T == 0, "a line's threads are in one wave");
    const uint32_t row0 = lg << n2;
    const uint32_t srow = aut_eval_src(row0, g, n) >> n2;
    const ulonglong2 *s2 = reinterpret_cast<const ulonglong2 *>(src + ((size_t)srow << n2) + E * t);
    ulonglong2 v[E / 2];
#pragma unroll
    for (int c = 0; c < E / 2; ++c) v[c] = s2[c];
#pragma unroll
    for (int c = 0; c < E / 2; ++c) {
        lds[TL::idx(line, E * t + 2 * c)] = v[c].x;
        lds[TL::idx(line, E * t + 2 * c + 1)] = v[c].y;
    }
    wave_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t k = k_of<IOL::IN_LO, IOL::IN_HI, E>(t, e);
        const uint32_t col = aut_eval_src(row0 + k, g, n) & ((1u << LOGS) - 1u);
        x[e] = lds[TL::idx(line, col)];
    }
    wave_sync();
}

struct NttArgs {
    const Ctx *ctx;  // host-side only (timing); not read by kernels
    const Shoup *tw;      // [M][N] forward or inverse table
    const uint64_t *twm;  // [M][N] the same table in Montgomery form (row passes)
    const ModC *mc;
    const LastInv *li;    // folded last inverse stage, indexed by cidx
    const Shoup *pinv;    // IO_MDEPI: P^-1 mod q_i
    uint32_t n, n1, n2, L;
    uint32_t nb;          // batch entries in blockIdx.x (xcd_batch) or blockIdx.y
    uint32_t xcd_batch;   // the entries of one (limb, tile) on one XCD, one after another
    LimbMap m;
    BatchIo io;
};

enum { IO_PLAIN = 0, IO_GATHER = 1, IO_REDUCE = 2, IO_MDEPI = 4, IO_MIXED = 8 };

template <int LOGS, int LINES, bool COLS, bool FWD, int IO, int E>
__global__ void __launch_bounds__((Tile<LOGS, LINES, COLS, E>::NT)) ntt_pass_kernel(const NttArgs a) {
    constexpr int IOB = IO & 7;
    constexpr bool MIXED = (IO & IO_MIXED) != 0;
    using TL = Tile<LOGS, LINES, COLS, E>;
    using IOL = IoLayout<LOGS, FWD, E>;
    __shared__ uint64_t lds[TL::WORDS];
    const uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
    const uint32_t tiles = lines_per_limb / LINES;
    // xcd_batch: block ids are dealt round-robin over the 8 XCDs, so the nb
    // entries of one (limb, tile) get ids equal modulo 8 and consecutive in
    // dispatch order: the second entry finds the tile's twiddles in L2
    uint32_t bx, b;
    if (a.xcd_batch) {
        const uint32_t rest = blockIdx.x >> 3;
        b = rest % a.nb;
        bx = ((rest / a.nb) << 3) | (blockIdx.x & 7u);
    } else {
        bx = blockIdx.x;
        b = blockIdx.y;
    }
    const uint32_t li = bx / tiles;
    const uint32_t tile = bx % tiles;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = a.m.mod[li];
    if constexpr (MIXED) {
        // an entry below the step's top level has no limb of the q primes at
        // or above its level, nor of the digits at or above its digit count
        const uint32_t lv = a.io.lvl[b], nbt = a.io.nbeta[b], dg = a.m.dig[li];
        if ((lv && mod < a.L && mod >= lv) || (nbt && dg != NO_DIGIT && dg >= nbt)) return;
    }
    const ModC mcv = a.mc[mod];
    const uint64_t q = mcv.q;
    const uint64_t *src = a.io.in[b] + (size_t)a.m.in_off[li] * N;
    uint64_t *dst = a.io.out[b] + (size_t)a.m.out_off[li] * N;
    const Shoup *tw = a.tw + (size_t)mod * N;
    int line, t;
    thread_coords<LOGS, LINES, COLS, E>(threadIdx.x, line, t);
    const uint32_t lg = tile * LINES + line;  // this thread's column or row

    // ModDown epilogue operands (u, and the automorphed addend), issued
    // before the pass input: loads complete in issue order, so one memory
    // latency covers all three instead of a second one after the pass
    uint64_t uv[E], bv[E];
    const uint32_t ui = a.m.cidx[li];
    const uint64_t *ad = (IOB == IO_MDEPI && a.io.add[b]) ? a.io.add[b] + (size_t)ui * N : nullptr;
    if (IOB == IO_MDEPI) {
        gload<LOGS, COLS, IOL::OUT_LO, IOL::OUT_HI, E>(uv, a.io.uq[b] + (size_t)ui * N, t, lg, a.n2);
        if (ad) {
            const uint32_t ag = a.io.add_galois[b];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t j = jdx<COLS>(lg, k_of<IOL::OUT_LO, IOL::OUT_HI, E>(t, e), a.n2);
                bv[e] = ad[ag != 1 ? aut_eval_src(j, ag, a.n) : j];
            }
        }
    }

    uint64_t x[E];
    if (IOB == IO_GATHER && !COLS) {
        gather_row<LOGS, LINES, FWD, E>(x, src, lds, line, t, lg, a.io.galois[b], a.n, a.n2);
    } else if (IOB == IO_GATHER) {
        const uint32_t g = a.io.galois[b];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t j = jdx<COLS>(lg, k_of<IOL::IN_LO, IOL::IN_HI, E>(t, e), a.n2);
            x[e] = src[g != 1 ? aut_eval_src(j, g, a.n) : j];
        }
    } else {
        gload<LOGS, COLS, IOL::IN_LO, IOL::IN_HI, E>(x, src, t, lg, a.n2);
    }

    const LastInv fold = (!FWD && COLS) ? a.li[a.m.cidx[li] + (MIXED ? a.io.cbase[b] : 0u)] : LastInv{};
    if constexpr (COLS) {
        pass_regs<LOGS, LINES, COLS, FWD, TW_HOIST, E, TW_PRE_COLS>(true, x, lds, line, t, q, mcv.nq, TwCols{tw},
                                                                    fold);
    } else if constexpr (MONT_ROWS<LOGS>) {
        pass_regs<LOGS, LINES, COLS, FWD, TW_HOIST, E, TW_PRE_ROWS>(
            true, x, lds, line, t, q, mcv.nq, TwRowsM{a.twm + (size_t)mod * N, lg, a.n1}, fold, mcv.qi);
    } else {
        pass_regs<LOGS, LINES, COLS, FWD, TW_HOIST, E, TW_PRE_ROWS>(true, x, lds, line, t, q, mcv.nq,
                                                                    TwRows{tw, lg, a.n1}, fold);
    }

    if (IOB == IO_MDEPI) {
        const Shoup pi = a.pinv[ui];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint64_t z = reduce64(x[e], q, mcv.mu, mcv.nq);
            uint64_t r = mul_shoup(uv[e] + q - z, pi.w, pi.wp, q);
            if (ad) r = add_mod(r, bv[e], q);
            x[e] = r;
        }
    } else if (IOB == IO_REDUCE) {
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = reduce64(x[e], q, mcv.mu, mcv.nq);
    }
    gstore<LOGS, COLS, IOL::OUT_LO, IOL::OUT_HI, E>(x, dst, t, lg, a.n2);
}

constexpr int COL_LINES = 16;  // columns per column-pass block (the default plan)
constexpr int ROW_LINES = 8;   // rows per row-pass block (the default plan)

// One pass launch: count limbs of `batch` entries, LINES lines per block.
template <int LOGS, bool COLS, bool FWD, int IO, int E, int LINES>
static hipError_t launch_pass_t(const NttArgs &a, uint32_t count, uint32_t batch, hipStream_t s) {
    using TL = Tile<LOGS, LINES, COLS, E>;
    if constexpr (TL::NT > 1024 || (1 << LOGS) / E < 1) {
        return hipErrorInvalidValue;
    } else {
        ProfScope ps(*a.ctx, FWD ? (COLS ? HKS_K_NTT_FWD_COLS : HKS_K_NTT_FWD_ROWS)
                                 : (COLS ? HKS_K_NTT_INV_COLS : HKS_K_NTT_INV_ROWS), s);
        const uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
        if (lines_per_limb < (uint32_t)LINES) return hipErrorInvalidValue;
        const uint32_t xs = count * (lines_per_limb / LINES);
        NttArgs ab = a;
        ab.nb = batch;
        // row passes read a twiddle table as large as the limb: share it
        // across the batch through L2 (column-pass twiddles are few and
        // always cached)
        ab.xcd_batch = (!COLS && batch > 1 && xs % 8 == 0 && a.ctx->plan.row_xcd_order) ? 1u : 0u;
        const dim3 grid = ab.xcd_batch ? dim3(xs * batch, 1) : dim3(xs, batch);
        hipLaunchKernelGGL((ntt_pass_kernel<LOGS, LINES, COLS, FWD, IO, E>), grid, dim3(TL::NT), 0, s, ab);
        return hipGetLastError();
    }
}

// A pass launch by run-time shape (ntt_cols.hip, ntt_rows_fwd.hip,
// ntt_rows_inv.hip instantiate the kernels): `io` is one of the IO modes
// the pass class uses, e 8 or 16 elements per thread, logs 5..9 stages,
// `lines` per block (8, 16 or 32 columns; 4, 8 or 16 rows; 7 <= logs only,
// the defaults elsewhere).  hipErrorInvalidValue for a shape not built.
hipError_t launch_pass_cols(const NttArgs &a, bool fwd, int io, int e, int logs, int lines, uint32_t count,
                            uint32_t batch, hipStream_t s);
hipError_t launch_pass_rows_fwd(const NttArgs &a, int io, int e, int logs, int lines, uint32_t count,
                                uint32_t batch, hipStream_t s);
hipError_t launch_pass_rows_inv(const NttArgs &a, int io, int e, int logs, int lines, uint32_t count,
                                uint32_t batch, hipStream_t s);

}  // namespace hks
