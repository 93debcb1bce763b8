// Negacyclic NTT / iNTT passes for gfx950 (Sec. 2.3) and the kernels that
// fuse key-switching steps into them.
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
// The butterflies of one phase on the thread's E registers (layout [LO, HI)).
// Each stage loads E >> (vb+1) distinct twiddles.  With FOLD (the inverse
// column pass) the global last inverse stage multiplies by the folded
// constants instead.
template <int LOGS, bool FWD, bool FOLD, int LO, int HI, bool HOIST, int E, typename TW>
__device__ __forceinline__ void phase_regs(uint64_t (&x)[E], int t, uint64_t q, uint64_t nq, const TW &tws,
                                           const LastInv &fold) {
    constexpr int B = HI - LO, H = E / 2;
    const uint64_t q2 = 2 * q;
    // HOIST: every twiddle of the phase loaded up front (E >> (vb+1) per
    // stage), one memory latency per phase instead of one per stage, for
    // more registers
    Shoup wall[HOIST ? B : 1][H];
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
        Shoup wc[H];
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
            const Shoup w = wc[(e >> (vb + 1)) & (H - 1)];
            if (FWD) {
                const uint64_t u = x[e];
                const uint64_t tv = mul_shoup_lazy_nq(x[e2], w.w, w.wp, nq);
                x[e] = u + tv;
                x[e2] = u + q2 - tv;
            } else {
                const uint64_t u = x[e], v = x[e2];
                if (fold_stage) {
                    x[e] = mul_shoup(u + v, fold.c.w, fold.c.wp, q);
                    x[e2] = mul_shoup(u + q2 - v, fold.cw.w, fold.cw.wp, q);
                } else {
                    x[e] = csub(u + v, q2);
                    x[e2] = mul_shoup_lazy_nq(u + q2 - v, w.w, w.wp, nq);
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
template <int LOGS, int LINES, bool COLS, bool FWD, bool HOIST, int E = 16, typename TW>
__device__ __forceinline__ void pass_regs(bool active, uint64_t (&x)[E], uint64_t *lds, int line, int t, uint64_t q,
                                          uint64_t nq, const TW &tws, const LastInv &fold) {
    using P = Phases<LOGS, Log2<E>::value>;
    constexpr bool FOLD = !FWD && COLS;
    if (FWD) {
        if (active) {
            phase_regs<LOGS, true, FOLD, P::P0L, P::P0H, HOIST, E>(x, t, q, nq, tws, fold);
            lds_put<LOGS, LINES, COLS, P::P0L, P::P0H, E>(lds, x, line, t);
        }
        __syncthreads();
        if (active) {
            lds_get<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            phase_regs<LOGS, true, FOLD, P::P1L, P::P1H, HOIST, E>(x, t, q, nq, tws, fold);
        }
        if constexpr (P::THREE) {
            __syncthreads();
            if (active) lds_put<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            __syncthreads();
            if (active) {
                lds_get<LOGS, LINES, COLS, P::P2L, P::P2H, E>(lds, x, line, t);
                phase_regs<LOGS, true, FOLD, P::P2L, P::P2H, HOIST, E>(x, t, q, nq, tws, fold);
            }
        }
    } else {
        if constexpr (P::THREE) {
            if (active) {
                phase_regs<LOGS, false, FOLD, P::P2L, P::P2H, HOIST, E>(x, t, q, nq, tws, fold);
                lds_put<LOGS, LINES, COLS, P::P2L, P::P2H, E>(lds, x, line, t);
            }
            __syncthreads();
            if (active) lds_get<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
            __syncthreads();
        }
        if (active) {
            phase_regs<LOGS, false, FOLD, P::P1L, P::P1H, HOIST, E>(x, t, q, nq, tws, fold);
            lds_put<LOGS, LINES, COLS, P::P1L, P::P1H, E>(lds, x, line, t);
        }
        __syncthreads();
        if (active) {
            lds_get<LOGS, LINES, COLS, P::P0L, P::P0H, E>(lds, x, line, t);
            phase_regs<LOGS, false, FOLD, P::P0L, P::P0H, HOIST, E>(x, t, q, nq, tws, fold);
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

struct NttArgs {
    const Ctx *ctx;  // host-side only (timing); not read by kernels
    const Shoup *tw;      // [M][N] forward or inverse table
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

// Whether the entries of a launch sit at different levels (per-entry limb
// limits or constant offsets set): only then do its blocks test whether their
// entry has their limb.
static bool io_mixed(const BatchIo &io, uint32_t batch) {
    for (uint32_t b = 0; b < batch && b < (uint32_t)MAXB; ++b)
        if (io.lvl[b] || io.nbeta[b] || io.cbase[b]) return true;
    return false;
}

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
    if (IOB == IO_GATHER) {
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
        pass_regs<LOGS, LINES, COLS, FWD, TW_HOIST, E>(true, x, lds, line, t, q, mcv.nq, TwCols{tw}, fold);
    } else {
        pass_regs<LOGS, LINES, COLS, FWD, TW_HOIST, E>(true, x, lds, line, t, q, mcv.nq, TwRows{tw, lg, a.n1}, fold);
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

constexpr int COL_LINES = 16;
constexpr int ROW_LINES = 8;

template <int LOGS, bool COLS, bool FWD, int IO, int E>
static hipError_t launch_pass_t(const NttArgs &a, uint32_t count, uint32_t batch, hipStream_t s) {
    constexpr int LINES = COLS ? COL_LINES : ROW_LINES;
    using TL = Tile<LOGS, LINES, COLS, E>;
    ProfScope ps(*a.ctx, FWD ? (COLS ? HKS_K_NTT_FWD_COLS : HKS_K_NTT_FWD_ROWS)
                             : (COLS ? HKS_K_NTT_INV_COLS : HKS_K_NTT_INV_ROWS), s);
    const uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
    const uint32_t xs = count * (lines_per_limb / LINES);
    NttArgs ab = a;
    ab.nb = batch;
    // row passes read a twiddle table as large as the limb: share it across
    // the batch through L2 (column-pass twiddles are few and always cached)
    ab.xcd_batch = (!COLS && batch > 1 && xs % 8 == 0 && a.ctx->plan.row_xcd_order) ? 1u : 0u;
    const dim3 grid = ab.xcd_batch ? dim3(xs * batch, 1) : dim3(xs, batch);
    hipLaunchKernelGGL((ntt_pass_kernel<LOGS, LINES, COLS, FWD, IO, E>), grid, dim3(TL::NT), 0, s, ab);
    return hipGetLastError();
}

// Elements per thread: 16 (radix-16 phases) when the launch has enough
// waves to fill the chip several times over (the plan's threshold for the
// pass class: 6 waves per SIMD by default, never for the forward row pass
// by default), else 8 (radix-8 phases, one more LDS exchange, twice the
// waves with half the work each), so that a small launch still hides its
// memory latency.

template <bool COLS, bool FWD, int IO, int E>
static hipError_t dispatch_pass_e(const NttArgs &a, int logs, uint32_t count, uint32_t batch, hipStream_t s) {
    switch (logs) {
        case 5: return launch_pass_t<5, COLS, FWD, IO, E>(a, count, batch, s);
        case 6: return launch_pass_t<6, COLS, FWD, IO, E>(a, count, batch, s);
        case 7: return launch_pass_t<7, COLS, FWD, IO, E>(a, count, batch, s);
        case 8: return launch_pass_t<8, COLS, FWD, IO, E>(a, count, batch, s);
        default: return hipErrorInvalidValue;
    }
}

template <bool COLS, bool FWD, int IO>
static hipError_t dispatch_pass_m(const NttArgs &a, int logs, uint32_t count, uint32_t batch, hipStream_t s) {
    const uint64_t waves16 = (uint64_t)count * batch * ((1ull << a.n) / 16) / 64;
    const int cls = FWD ? (COLS ? HKS_K_NTT_FWD_COLS : HKS_K_NTT_FWD_ROWS)
                        : (COLS ? HKS_K_NTT_INV_COLS : HKS_K_NTT_INV_ROWS);
    return waves16 >= a.ctx->plan.e16_min_waves[cls] ? dispatch_pass_e<COLS, FWD, IO, 16>(a, logs, count, batch, s)
                                                     : dispatch_pass_e<COLS, FWD, IO, 8>(a, logs, count, batch, s);
}

template <bool COLS, bool FWD, int IO>
static hipError_t dispatch_pass(const NttArgs &a, int logs, uint32_t count, uint32_t batch, hipStream_t s) {
    if (count == 0 || batch == 0) return hipSuccess;
    if (batch > (uint32_t)MAXB) return hipErrorInvalidValue;
    // the forward row pass with a reduced output serves whole transforms
    // (never a mixed-level step)
    if constexpr (IO != IO_REDUCE) {
        if (io_mixed(a.io, batch)) return dispatch_pass_m<COLS, FWD, IO | IO_MIXED>(a, logs, count, batch, s);
    } else {
        if (io_mixed(a.io, batch)) return hipErrorInvalidValue;
    }
    return dispatch_pass_m<COLS, FWD, IO>(a, logs, count, batch, s);
}

static NttArgs base_args(const Ctx &c, const LimbMap &m, const BatchIo &io, bool fwd) {
    NttArgs a{};
    a.ctx = &c;
    a.tw = fwd ? c.tw_fwd : c.tw_inv;
    a.mc = c.mc;
    a.li = c.li_plain;
    a.pinv = c.pinv;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.L = c.L;
    a.m = m;
    a.io = io;
    return a;
}

// the second pass of a transform reads what the first wrote
static void chain(NttArgs &a, uint32_t batch) {
    for (uint32_t i = 0; i < a.m.count; ++i) a.m.in_off[i] = a.m.out_off[i];
    for (uint32_t b = 0; b < batch; ++b) {
        a.io.in[b] = a.io.out[b];
        a.io.galois[b] = 1;
    }
}

hipError_t launch_ntt_fwd(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    NttArgs a = base_args(c, m, io, true);
    hipError_t e = dispatch_pass<true, true, IO_PLAIN>(a, c.n1, m.count, batch, s);
    if (e != hipSuccess) return e;
    chain(a, batch);
    return dispatch_pass<false, true, IO_REDUCE>(a, c.n2, m.count, batch, s);
}

hipError_t launch_ntt_fwd_cols(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    return dispatch_pass<true, true, IO_PLAIN>(base_args(c, m, io, true), c.n1, m.count, batch, s);
}

hipError_t launch_ntt_fwd_rows(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    return dispatch_pass<false, true, IO_REDUCE>(base_args(c, m, io, true), c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv(const Ctx &c, const LimbMap &m, const BatchIo &io, const LastInv *li, uint32_t batch,
                          hipStream_t s) {
    NttArgs a = base_args(c, m, io, false);
    a.li = li;
    bool gather = false;
    for (uint32_t b = 0; b < batch && b < (uint32_t)MAXB; ++b) gather |= io.galois[b] != 1;
    hipError_t e = gather ? dispatch_pass<false, false, IO_GATHER>(a, c.n2, m.count, batch, s)
                          : dispatch_pass<false, false, IO_PLAIN>(a, c.n2, m.count, batch, s);
    if (e != hipSuccess) return e;
    chain(a, batch);
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

hipError_t launch_ntt_inv_rows(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    return dispatch_pass<false, false, IO_PLAIN>(base_args(c, m, io, false), c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv_cols(const Ctx &c, const LimbMap &m, const BatchIo &io, const LastInv *li,
                               uint32_t batch, hipStream_t s) {
    NttArgs a = base_args(c, m, io, false);
    a.li = li;
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

hipError_t launch_rows_mdepi(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, const Shoup *pinv,
                             hipStream_t s) {
    NttArgs a = base_args(c, m, io, true);
    a.pinv = pinv;
    return dispatch_pass<false, true, IO_MDEPI>(a, c.n2, m.count, batch, s);
}

// ------------------------------------------------------------------ KSKInnerProd (+ ModUp's last pass, + ModDown's first)

#ifndef KSK_E8_WAVES
#define KSK_E8_WAVES 2
#endif

struct KskRowArgs {
    KskBatch kb;             // per ciphertext: own-digit source, key [dnum][2][L+K][N], galois
    const uint64_t *ext;     // [beta][E][N] converted limbs: after the forward column pass (rowpass) or in evaluation form
    uint64_t *uq;            // [2][level][N] KSKInnerProd on the q limbs
    uint64_t *pc;            // [2][K][N] P limbs after the inverse row pass
    const Shoup *twf, *twi;
    const ModC *mc;
    const Shoup *pmod;  // NewMult: [P]_{q_i}
    size_t dstride, ext_bstride, uq_bstride, pc_bstride;
    uint32_t n, n1, n2, L, K, alpha, all_direct, keyidx, nb, xcd_group, pck;
    uint32_t level0, uniform;  // every entry at level0 (uniform), else kb.level[b]
};

// One block = one target limb t of Q_level U P and ROW_LINES rows, in the
// row-pass layout (each thread 16 elements of one row).  For each digit j:
// the converted limb x_{j,t} gets the forward row pass on chip (ROWPASS: the
// last pass of ModUp's NTT; lazy values < 2^56), or the digit's own limb is
// read from the input through the automorph; then u_t += x ksk[j][0][t],
// v_t += x ksk[j][1][t] (Barrett products of the lazy value and the key,
// canonical sums).  q limbs store (u_t, v_t); special-prime limbs run
// ModDown's inverse row pass on both in registers before storing (the
// forward pass ends in the layout the inverse pass starts from).
// (at least two waves per SIMD: the register budget stays within 256)
template <int LOGS, bool ROWPASS, int E, bool SEEDED, bool NM>
__global__ void __launch_bounds__((Tile<LOGS, ROW_LINES, false, E>::NT)) __attribute__((amdgpu_waves_per_eu(E == 8 ? KSK_E8_WAVES : 2)))
ksk_rows_kernel(const KskRowArgs a) {
    using TL = Tile<LOGS, ROW_LINES, false, E>;
    using IOF = IoLayout<LOGS, true, E>;
    using IOI = IoLayout<LOGS, false, E>;
    static_assert(IOF::OUT_LO == IOI::IN_LO && IOF::OUT_HI == IOI::IN_HI, "row-pass layouts must chain");
    __shared__ uint64_t lds[TL::WORDS];
    // direct digits (hoisted rotations): the special limbs' inverse row-pass
    // twiddles for the block's ROW_LINES rows (every stage), staged once for
    // u's and v's passes (measured: HRotate +2%; with the forward row passes
    // of ROWPASS the staging latency costs more than it saves)
    __shared__ Shoup lds_tw[ROWPASS ? 1 : ROW_LINES * ((1 << LOGS) - 1)];
    // block -> (x = target limb and row tile, b = ciphertext).  With
    // xcd_group the nb blocks of one x get ids that are equal modulo 8, so
    // that they run on one XCD (ids are dealt round-robin over the 8 XCDs)
    // and a shared key tile is fetched into that XCD's L2 once.
    uint32_t x, b;
    if (a.xcd_group) {
        const uint32_t rest = blockIdx.x >> 3;
        b = rest % a.nb;
        x = ((rest / a.nb) << 3) | (blockIdx.x & 7u);
    } else {
        b = blockIdx.x % a.nb;
        x = blockIdx.x / a.nb;
    }
    const uint32_t tiles = (1u << a.n1) / ROW_LINES;
    // the entry's level (entries of one step may differ): the grid covers
    // the step's largest Q_level U P, smaller entries leave the rest
    const uint32_t level = a.uniform ? a.level0 : a.kb.level[b], Eb = level + a.K;
    if (x / tiles >= Eb) return;
    const uint32_t beta = (level + a.alpha - 1) / a.alpha;
    // special-prime limbs first: their blocks also run ModDown's inverse row
    // passes, so they go out in the first wave of blocks rather than the tail
    const uint32_t tgt = (x / tiles + level) % Eb;
    const uint32_t tile = x % tiles;
    const uint32_t N = 1u << a.n;
    const uint64_t *ext = a.ext + b * a.ext_bstride;
    const uint64_t *direct = a.kb.direct[b];
    const uint64_t *ksk = a.kb.ksk[b];
    const uint64_t seed = a.kb.seed[b];
    const uint32_t galois = a.kb.galois[b];
    uint64_t *uq = a.uq + b * a.uq_bstride;
    uint64_t *pc = a.pc + b * a.pc_bstride;
    const uint32_t mod = tgt < level ? tgt : a.L + (tgt - level);
    const ModC mcv = a.mc[mod];
    const uint64_t q = mcv.q;
    const size_t KL = (size_t)a.L + a.K;
    const uint32_t own = (tgt < level) ? tgt / a.alpha : 0xffffffffu;
    // special limbs: the P limbs, and with NM also q_(level-1) (stored after them)
    const bool is_p = tgt >= level || (NM && tgt == level - 1);
    const uint32_t kp = tgt >= level ? tgt - level : a.K;
    // the converted limbs of this target: packed digits of E limbs, or
    // key-indexed digits of L + K limbs (the same slots at every level)
    const size_t ext_ds = a.keyidx ? KL : Eb, ext_slot = a.keyidx ? mod : tgt;
    int line, t;
    thread_coords<LOGS, ROW_LINES, false, E>(threadIdx.x, line, t);
    const uint32_t lg = tile * ROW_LINES + line;

    // KSKInnerProd sums: with LAZY (8 elements per thread, where the
    // registers allow) the digits' 128-bit products are added without
    // reduction (each < 2^106: row-pass outputs < 2^56 times key words
    // < 2^50) and reduced once, folding every 16 digits to stay below 2^111
    constexpr bool LAZY = E == 8;
    uint64_t u[E], v[E];
    Acc128 ua[LAZY ? E : 1], va[LAZY ? E : 1];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = v[e] = 0;
    bool lds_used = false;
    for (uint32_t jd = 0; jd < beta; ++jd) {
        if (LAZY && jd && (jd & 15) == 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                ua[LAZY ? e : 0] = Acc128(reduce128(ua[LAZY ? e : 0].hi, ua[LAZY ? e : 0].lo, q, mcv.mu, mcv.nq));
                va[LAZY ? e : 0] = Acc128(reduce128(va[LAZY ? e : 0].hi, va[LAZY ? e : 0].lo, q, mcv.mu, mcv.nq));
            }
        }
        const bool dir = a.all_direct || jd == own;
        uint64_t xv[E];
        if (dir) {
            const uint64_t *src = direct + jd * a.dstride + (size_t)tgt * N;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t j = jdx<false>(lg, k_of<IOF::OUT_LO, IOF::OUT_HI, E>(t, e), a.n2);
                xv[e] = src[galois != 1 ? aut_eval_src(j, galois, a.n) : j];
            }
        } else {
            const uint64_t *src = ext + (jd * ext_ds + ext_slot) * N;
            if (ROWPASS) {
                gload<LOGS, false, IOF::IN_LO, IOF::IN_HI, E>(xv, src, t, lg, a.n2);
                if (lds_used) __syncthreads();
                pass_regs<LOGS, ROW_LINES, false, true, false, E>(true, xv, lds, line, t, q, mcv.nq,
                                                        TwRows{a.twf + (size_t)mod * N, lg, a.n1}, LastInv{});
                lds_used = true;
            } else {
                gload<LOGS, false, IOF::OUT_LO, IOF::OUT_HI, E>(xv, src, t, lg, a.n2);
            }
        }
        // the key rows in the same layout: E consecutive words per thread
        // (slots (lg << n2) + E t + e); a seeded key stores only the rows b_j
        // and regenerates a_j
        static_assert(IOF::OUT_LO == 0, "forward row pass ends with E consecutive elements per thread");
        const uint32_t slot0 = (lg << a.n2) + E * t;
        const ulonglong2 *k0 =
            reinterpret_cast<const ulonglong2 *>(ksk + ((size_t)(2 * jd) * KL + mod) * N + slot0);
        const ulonglong2 *k1 = SEEDED
            ? reinterpret_cast<const ulonglong2 *>(ksk + ((size_t)jd * KL + mod) * N + slot0)
            : k0 + KL * N / 2;
#pragma unroll
        for (int c = 0; c < E / 2; ++c) {
            ulonglong2 kv0;
            if constexpr (SEEDED) {
                kv0.x = seeded_key_a(seed, jd, mod, slot0 + 2 * c, q, mcv.mu, mcv.nq);
                kv0.y = seeded_key_a(seed, jd, mod, slot0 + 2 * c + 1, q, mcv.mu, mcv.nq);
            } else {
                kv0 = k0[c];
            }
            const ulonglong2 kv1 = k1[c];
            if constexpr (LAZY) {
                ua[2 * c].mac(xv[2 * c], kv0.x);
                ua[2 * c + 1].mac(xv[2 * c + 1], kv0.y);
                va[2 * c].mac(xv[2 * c], kv1.x);
                va[2 * c + 1].mac(xv[2 * c + 1], kv1.y);
            } else {
                u[2 * c] = add_mod(u[2 * c], mul_mod(xv[2 * c], kv0.x, q, mcv.mu, mcv.nq), q);
                u[2 * c + 1] = add_mod(u[2 * c + 1], mul_mod(xv[2 * c + 1], kv0.y, q, mcv.mu, mcv.nq), q);
                v[2 * c] = add_mod(v[2 * c], mul_mod(xv[2 * c], kv1.x, q, mcv.mu, mcv.nq), q);
                v[2 * c + 1] = add_mod(v[2 * c + 1], mul_mod(xv[2 * c + 1], kv1.y, q, mcv.mu, mcv.nq), q);
            }
        }
    }
    if constexpr (LAZY) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            u[e] = reduce128(ua[LAZY ? e : 0].hi, ua[LAZY ? e : 0].lo, q, mcv.mu, mcv.nq);
            v[e] = reduce128(va[LAZY ? e : 0].hi, va[LAZY ? e : 0].lo, q, mcv.mu, mcv.nq);
        }
    }
    if constexpr (NM) {
        // NewMult: u += P b3, v += P c3 on the q limbs (PModUp)
        if (tgt < level) {
            const Shoup pm = a.pmod[tgt];
            const uint64_t *b3 = a.kb.addp[b] + (size_t)tgt * N + (lg << a.n2) + E * t;
            const uint64_t *c3 = b3 + (size_t)level * N;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                u[e] = add_mod(u[e], mul_shoup(b3[e], pm.w, pm.wp, q), q);
                v[e] = add_mod(v[e], mul_shoup(c3[e], pm.w, pm.wp, q), q);
            }
        }
    }
    if (!is_p) {
        gstore<LOGS, false, IOF::OUT_LO, IOF::OUT_HI, E>(u, uq + (size_t)tgt * N, t, lg, a.n2);
        gstore<LOGS, false, IOF::OUT_LO, IOF::OUT_HI, E>(v, uq + ((size_t)level + tgt) * N, t, lg, a.n2);
        return;
    }
    // special limb: inverse row pass (first pass of ModDown's iNTT) of u and v
    if (lds_used) __syncthreads();
    if constexpr (ROWPASS) {
        const TwRows twi{a.twi + (size_t)mod * N, lg, a.n1};
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, u, lds, line, t, q, mcv.nq, twi, LastInv{});
        gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(u, pc + (size_t)kp * N, t, lg, a.n2);
        __syncthreads();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, v, lds, line, t, q, mcv.nq, twi, LastInv{});
    } else {
        const TwRowsLds<ROW_LINES> twl{lds_tw, (uint32_t)line};
        stage_row_twiddles<LOGS, ROW_LINES>(lds_tw, a.twi + (size_t)mod * N, tile * ROW_LINES, a.n1);
        __syncthreads();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, u, lds, line, t, q, mcv.nq, twl, LastInv{});
        gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(u, pc + (size_t)kp * N, t, lg, a.n2);
        __syncthreads();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, v, lds, line, t, q, mcv.nq, twl, LastInv{});
    }
    gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(v, pc + ((size_t)a.pck + kp) * N, t, lg, a.n2);
}

template <bool ROWPASS, int E, bool SEEDED, bool NM = false>
static hipError_t launch_ksk_rows_t(const KskRowArgs &a, uint32_t n2, dim3 grid, hipStream_t s) {
    switch (n2) {
        case 5: hipLaunchKernelGGL((ksk_rows_kernel<5, ROWPASS, E, SEEDED, NM>), grid, dim3(Tile<5, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 6: hipLaunchKernelGGL((ksk_rows_kernel<6, ROWPASS, E, SEEDED, NM>), grid, dim3(Tile<6, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 7: hipLaunchKernelGGL((ksk_rows_kernel<7, ROWPASS, E, SEEDED, NM>), grid, dim3(Tile<7, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 8: hipLaunchKernelGGL((ksk_rows_kernel<8, ROWPASS, E, SEEDED, NM>), grid, dim3(Tile<8, ROW_LINES, false, E>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ksk_rows(const Ctx &c, const KskBatch &kb, uint32_t nb, const uint64_t *ext, size_t ext_bstride,
                           bool rowpass, bool keyidx, size_t dstride, uint32_t all_direct, uint64_t *uq,
                           size_t uq_bstride, uint64_t *pc, size_t pc_bstride, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    if (nb > (uint32_t)MAXCT) return hipErrorInvalidValue;
    uint32_t top = 0;
    bool uniform = true;
    for (uint32_t b = 0; b < nb; ++b) {
        if (kb.level[b] < 1 || kb.level[b] > c.L) return hipErrorInvalidValue;
        top = std::max(top, kb.level[b]);
        uniform = uniform && kb.level[b] == kb.level[0];
    }
    KskRowArgs a{};
    a.level0 = kb.level[0];
    a.uniform = uniform ? 1u : 0u;
    a.kb = kb;
    a.ext = ext;
    a.ext_bstride = ext_bstride;
    a.dstride = dstride;
    a.all_direct = all_direct;
    a.uq = uq;
    a.uq_bstride = uq_bstride;
    a.pc = pc;
    a.pc_bstride = pc_bstride;
    a.twf = c.tw_fwd;
    a.twi = c.tw_inv;
    a.mc = c.mc;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.L = c.L;
    a.K = c.K;
    a.alpha = c.alpha;
    a.keyidx = keyidx ? 1u : 0u;
    a.nb = nb;
    a.pmod = c.pmod;
    a.pck = kb.newmult ? c.K + 1 : c.K;
    // (target limb, row tile) items of the step's largest entry
    const uint32_t xs = ((1u << c.n1) / ROW_LINES) * (top + c.K);
    a.xcd_group = (nb > 1 && xs % 8 == 0 && c.plan.ksk_xcd_order) ? 1u : 0u;
    ProfScope ps(c, HKS_K_KSK, s);
    const dim3 grid(xs * nb);
    // 8 elements per thread for every launch: the 128-bit lazy sums fit in
    // the registers only there, and measured faster than 16 also for
    // batched and hoisted launches
    if (kb.newmult) {  // NewMult: a relinearization key, the converted limbs after the column pass
        if (!rowpass || kb.seeded) return hipErrorInvalidValue;
        return launch_ksk_rows_t<true, 8, false, true>(a, c.n2, grid, s);
    }
    // a seeded key's rows a_j are generated in the kernel
    if (kb.seeded)
        return rowpass ? launch_ksk_rows_t<true, 8, true>(a, c.n2, grid, s)
                       : launch_ksk_rows_t<false, 8, true>(a, c.n2, grid, s);
    return rowpass ? launch_ksk_rows_t<true, 8, false>(a, c.n2, grid, s)
                   : launch_ksk_rows_t<false, 8, false>(a, c.n2, grid, s);
}

// ------------------------------------------------------------------ PtMatVecMult with one ModDown

struct MatvecArgs {
    const uint64_t *ext;  // [beta][E][N] extended digits of a_x, evaluation form
    const uint64_t *ax;   // a_x, [level][N] (the diagonal without rotation)
    const uint64_t *ksk[MAXROT];  // nullptr: the diagonal without rotation (g = 1)
    const uint64_t *pt[MAXROT];  // diagonals over Q_level U P, [level + K][N]
    uint32_t galois[MAXROT];
    const uint64_t *b;     // b_x, [level][N]
    const Shoup *pmod;     // [P]_{q_i}
    uint64_t *uq;          // [2][level][N] sums on the q limbs
    uint64_t *pc;          // [2][K][N] sums on the P limbs after the inverse row pass
    const Shoup *twi;
    const ModC *mc;
    uint32_t n, n1, n2, level, L, K, E, beta, r;
};

// One block = one limb t of Q_level U P and ROW_LINES rows, over all r
// rotations (the paper's PtMatVecMult with the ModDown hoisted): for each i,
// u, v = KSKInnerProd of the extended digits gathered through g_i with
// ksk_i; then a_y += M_i u and b_y += M_i (v + [P]_t b_rot) where b_rot is b
// gathered through g_i (q limbs only).  A term without a key is the diagonal
// of offset 0: (u, v) = ([P]_t a_x, 0) on the q limbs, 0 on the P limbs
// (PModUp of the input, no key switch).  The sums stay in registers; q limbs
// store them, P limbs run ModDown's inverse row pass first.
template <int LOGS, int E>
__global__ void __launch_bounds__((Tile<LOGS, ROW_LINES, false, E>::NT)) ksk_matvec_kernel(const MatvecArgs a) {
    using TL = Tile<LOGS, ROW_LINES, false, E>;
    using IOF = IoLayout<LOGS, true, E>;
    using IOI = IoLayout<LOGS, false, E>;
    static_assert(IOF::OUT_LO == 0 && IOF::OUT_LO == IOI::IN_LO && IOF::OUT_HI == IOI::IN_HI,
                  "E consecutive slots per thread, the inverse row pass's input layout");
    __shared__ uint64_t lds[TL::WORDS];
    const uint32_t tiles = (1u << a.n1) / ROW_LINES;
    const uint32_t tgt = (blockIdx.x / tiles + a.level) % a.E;  // special-prime limbs first
    const uint32_t tile = blockIdx.x % tiles;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = tgt < a.level ? tgt : a.L + (tgt - a.level);
    const ModC mcv = a.mc[mod];
    const uint64_t q = mcv.q;
    const size_t KL = (size_t)a.L + a.K;
    const bool is_p = tgt >= a.level;
    int line, t;
    thread_coords<LOGS, ROW_LINES, false, E>(threadIdx.x, line, t);
    const uint32_t lg = tile * ROW_LINES + line;
    const uint32_t slot0 = (lg << a.n2) + E * t;
    const Shoup pm = is_p ? Shoup{} : a.pmod[tgt];

    uint64_t ya[E], yb[E];
#pragma unroll
    for (int e = 0; e < E; ++e) ya[e] = yb[e] = 0;
    for (uint32_t i = 0; i < a.r; ++i) {
        const uint32_t g = a.galois[i];
        uint64_t u[E], v[E];
        // the digits' products (canonical times canonical, < 2^100) summed in
        // 128 bits and reduced once per rotation (beta < 2^11 keeps the sum
        // below Barrett's 2^111 bound)
        Acc128 ua[E], va[E];
#pragma unroll
        for (int e = 0; e < E; ++e) u[e] = v[e] = 0;
        if (!a.ksk[i]) {
            if (!is_p) {
                const ulonglong2 *ar = reinterpret_cast<const ulonglong2 *>(a.ax + (size_t)tgt * N + slot0);
#pragma unroll
                for (int c = 0; c < E / 2; ++c) {
                    const ulonglong2 x = ar[c];
                    u[2 * c] = mul_shoup(x.x, pm.w, pm.wp, q);
                    u[2 * c + 1] = mul_shoup(x.y, pm.w, pm.wp, q);
                }
            }
        }
        for (uint32_t jd = 0; a.ksk[i] && jd < a.beta; ++jd) {
            const uint64_t *src = a.ext + ((size_t)jd * a.E + tgt) * N;
            const ulonglong2 *k0 =
                reinterpret_cast<const ulonglong2 *>(a.ksk[i] + ((size_t)(2 * jd) * KL + mod) * N + slot0);
            const ulonglong2 *k1 = k0 + KL * N / 2;
#pragma unroll
            for (int c = 0; c < E / 2; ++c) {
                const ulonglong2 kv0 = k0[c], kv1 = k1[c];
                const uint64_t x0 = src[aut_eval_src(slot0 + 2 * c, g, a.n)];
                const uint64_t x1 = src[aut_eval_src(slot0 + 2 * c + 1, g, a.n)];
                ua[2 * c].mac(x0, kv0.x);
                ua[2 * c + 1].mac(x1, kv0.y);
                va[2 * c].mac(x0, kv1.x);
                va[2 * c + 1].mac(x1, kv1.y);
            }
        }
        if (a.ksk[i]) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                u[e] = reduce128(ua[e].hi, ua[e].lo, q, mcv.mu, mcv.nq);
                v[e] = reduce128(va[e].hi, va[e].lo, q, mcv.mu, mcv.nq);
            }
        }
        const ulonglong2 *mi = reinterpret_cast<const ulonglong2 *>(a.pt[i] + (size_t)tgt * N + slot0);
        const uint64_t *brow = a.b + (size_t)tgt * N;
#pragma unroll
        for (int c = 0; c < E / 2; ++c) {
            const ulonglong2 m = mi[c];
            uint64_t v0 = v[2 * c], v1 = v[2 * c + 1];
            if (!is_p) {
                v0 = add_mod(v0, mul_shoup(brow[aut_eval_src(slot0 + 2 * c, g, a.n)], pm.w, pm.wp, q), q);
                v1 = add_mod(v1, mul_shoup(brow[aut_eval_src(slot0 + 2 * c + 1, g, a.n)], pm.w, pm.wp, q), q);
            }
            ya[2 * c] = add_mod(ya[2 * c], mul_mod(m.x, u[2 * c], q, mcv.mu, mcv.nq), q);
            ya[2 * c + 1] = add_mod(ya[2 * c + 1], mul_mod(m.y, u[2 * c + 1], q, mcv.mu, mcv.nq), q);
            yb[2 * c] = add_mod(yb[2 * c], mul_mod(m.x, v0, q, mcv.mu, mcv.nq), q);
            yb[2 * c + 1] = add_mod(yb[2 * c + 1], mul_mod(m.y, v1, q, mcv.mu, mcv.nq), q);
        }
    }
    if (!is_p) {
        gstore<LOGS, false, IOF::OUT_LO, IOF::OUT_HI, E>(ya, a.uq + (size_t)tgt * N, t, lg, a.n2);
        gstore<LOGS, false, IOF::OUT_LO, IOF::OUT_HI, E>(yb, a.uq + ((size_t)a.level + tgt) * N, t, lg, a.n2);
        return;
    }
    const uint32_t kp = tgt - a.level;
    const TwRows twi{a.twi + (size_t)mod * N, lg, a.n1};
    pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, ya, lds, line, t, q, mcv.nq, twi, LastInv{});
    gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(ya, a.pc + (size_t)kp * N, t, lg, a.n2);
    __syncthreads();
    pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, yb, lds, line, t, q, mcv.nq, twi, LastInv{});
    gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(yb, a.pc + ((size_t)a.K + kp) * N, t, lg, a.n2);
}

hipError_t launch_ksk_matvec(const Ctx &c, const uint64_t *ext, uint32_t level, uint32_t r, const uint32_t *galois,
                             const uint64_t *const *ksk, const uint64_t *const *pt, const uint64_t *ax,
                             const uint64_t *b, uint64_t *uq, uint64_t *pc, hipStream_t s) {
    if (r == 0 || r > (uint32_t)MAXROT) return hipErrorInvalidValue;
    MatvecArgs a{};
    a.ext = ext;
    a.ax = ax;
    for (uint32_t i = 0; i < r; ++i) {
        a.ksk[i] = ksk[i];
        a.pt[i] = pt[i];
        a.galois[i] = galois[i];
    }
    a.b = b;
    a.pmod = c.pmod;
    a.uq = uq;
    a.pc = pc;
    a.twi = c.tw_inv;
    a.mc = c.mc;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.level = level;
    a.L = c.L;
    a.K = c.K;
    a.E = level + c.K;
    a.beta = (level + c.alpha - 1) / c.alpha;
    a.r = r;
    ProfScope ps(c, HKS_K_KSK, s);
    const dim3 grid(((1u << c.n1) / ROW_LINES) * a.E);
    switch (c.n2) {
        case 5: hipLaunchKernelGGL((ksk_matvec_kernel<5, 8>), grid, dim3(Tile<5, ROW_LINES, false, 8>::NT), 0, s, a); break;
        case 6: hipLaunchKernelGGL((ksk_matvec_kernel<6, 8>), grid, dim3(Tile<6, ROW_LINES, false, 8>::NT), 0, s, a); break;
        case 7: hipLaunchKernelGGL((ksk_matvec_kernel<7, 8>), grid, dim3(Tile<7, ROW_LINES, false, 8>::NT), 0, s, a); break;
        case 8: hipLaunchKernelGGL((ksk_matvec_kernel<8, 8>), grid, dim3(Tile<8, ROW_LINES, false, 8>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hks
