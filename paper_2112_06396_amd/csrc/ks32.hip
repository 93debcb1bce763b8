// Kernels of the 32-bit-word key-switch (Sec. 5.4).  Same structure as the
// 64-bit path: each NTT is a column pass (stages 0..n1-1) and a row pass
// (stages n1..n-1) over the 2^n1 x 2^n2 view of a limb, 16 elements per
// thread in registers with LDS exchanges between phases of four stages; the
// automorphism is gathered inside loads; KSKInnerProd runs inside the
// forward row pass of the extended limbs and goes on with ModDown's inverse
// row pass on the P limbs; ModDown's final step runs inside the last
// forward row pass.
//
// Arithmetic for primes q < 2^30 (so 4q < 2^32):
//   Shoup:      x w mod q = x w - floor(x w' / 2^32) q (mod 2^32), in [0, 2q),
//               for any 32-bit x (w' = floor(w 2^32 / q));
//   forward:    Harvey's butterfly on values in [0, 4q): u -> u mod 2q,
//               t = w x' in [0, 2q), (u + t, u - t + 2q);
//   inverse:    on values in [0, 2q): (u + v mod 2q, w (u - v + 2q));
//   sums:       products of canonical residues are < 2^60, so 16 of them
//               add exactly in a 64-bit word; one Barrett step with
//               mu = floor(2^64 / q) and two conditional subtractions reduce.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "ks32.h"

namespace hks {
namespace w32 {

constexpr int E32 = 16;        // elements per thread of the NTT passes
constexpr int EK32 = 16;       // elements per thread of the key-switch kernel (8 measured slower)
constexpr int COL32 = 32;      // columns per column tile (128-byte segments)
constexpr int ROW32 = 8;       // rows per row tile

template <int LOGS, int LINES, bool COLS, int E = E32>
struct Tile32 {
    static constexpr int S = 1 << LOGS;
    static constexpr int T = S / E;
    static constexpr int NT = LINES * T;
    static constexpr int ROWP = S + S / 32;
    static constexpr int COLP = LINES + 1;
    static constexpr int WORDS = COLS ? S * COLP : LINES * ROWP;
    __device__ static __forceinline__ int idx(int line, int k) {
        return COLS ? k * COLP + line : line * ROWP + k + (k >> 5);
    }
};

// Phases of R = log2(E) stages over the LOGS bits of the in-line index k:
// P0 = [LOGS-R, LOGS), P1 = [max(LOGS-2R, 0), LOGS-R), P2 = [0, LOGS-2R)
// when LOGS > 2R.  The forward pass runs P0, P1 (, P2); the inverse the
// reverse.  HL/HH is the high phase P0, LL/LH the lowest (P2, or P1).
template <int LOGS, int E = E32>
struct Ph32 {
    static constexpr int R = E == 16 ? 4 : 3;
    static_assert(E == 8 || E == 16, "8 or 16 elements per thread");
    static_assert(LOGS > R && LOGS <= 3 * R, "two or three phases");
    static constexpr bool THREE = LOGS > 2 * R;
    static constexpr int HL = LOGS - R, HH = LOGS;
    static constexpr int ML = THREE ? LOGS - 2 * R : 0, MH = LOGS - R;  // P1
    static constexpr int LL = 0, LH = THREE ? LOGS - 2 * R : LOGS - R;
};

// element e of thread t in the layout of phase [LO, HI) (see the 64-bit
// kernels: the thread holds all values of bits [LO, HI) for E >> (HI-LO)
// values of the other bits)
template <int LO, int HI, int E = E32>
__device__ __forceinline__ int k32(int t, int e) {
    constexpr int B = HI - LO, G = E >> B;
    const int v = e & ((1 << B) - 1), g = e >> B;
    const int r = t * G + g;
    return ((r >> LO) << HI) | (v << LO) | (r & ((1 << LO) - 1));
}

template <bool COLS>
__device__ __forceinline__ uint32_t jdx32(uint32_t lg, int k, uint32_t n2) {
    return COLS ? (((uint32_t)k << n2) + lg) : ((lg << n2) + (uint32_t)k);
}

__device__ __forceinline__ uint32_t shoup32(uint32_t x, uint32_t w, uint32_t wp, uint32_t q) {
    return x * w - __umulhi(x, wp) * q;
}
__device__ __forceinline__ uint32_t csub32(uint32_t x, uint32_t m) { return x >= m ? x - m : x; }

// x mod q for any 64-bit x: floor(x mu / 2^64) is at most two below
// floor(x / q), so the remainder is in [0, 3q) before two subtractions.
__device__ __forceinline__ uint32_t reduce64_32(uint64_t x, const Mod32 &m) {
    const uint64_t qh = __umul64hi(x, m.mu);
    const uint32_t r = (uint32_t)(x - qh * m.q);
    return csub32(csub32(r, 2 * m.q), m.q);
}

struct Tw32Cols {
    const Shoup32 *tw;
    __device__ __forceinline__ Shoup32 operator()(int ls, uint32_t mm) const { return tw[(1u << ls) + mm]; }
};
struct Tw32Rows {
    const Shoup32 *tw;
    uint32_t row, n1;
    __device__ __forceinline__ Shoup32 operator()(int ls, uint32_t mm) const {
        return tw[(((1u << n1) + row) << ls) + mm];
    }
};

template <int LOGS, bool FWD, bool FOLD, int LO, int HI, int E, typename TW>
__device__ __forceinline__ void phase32(uint32_t (&x)[E], int t, uint32_t q, const TW &tws, const Last32 &fold) {
    constexpr int B = HI - LO, H = E / 2;
    const uint32_t q2 = 2 * q;
#pragma unroll
    for (int st = 0; st < B; ++st) {
        const int bit = FWD ? (HI - 1 - st) : (LO + st);
        const int vb = bit - LO;
        const int ls = LOGS - 1 - bit;  // stage within this pass
        const bool fold_stage = FOLD && ls == 0;
        Shoup32 wc[H];
#pragma unroll
        for (int key = 0; key < H; ++key) {
            if (key < (E >> (vb + 1)) && !fold_stage) {
                const uint32_t k = (uint32_t)k32<LO, HI, E>(t, key << (vb + 1));
                wc[key] = tws(ls, k >> (bit + 1));
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if ((e >> vb) & 1) continue;
            const int e2 = e + (1 << vb);
            const Shoup32 w = wc[(e >> (vb + 1)) & (H - 1)];
            if (FWD) {
                const uint32_t u = csub32(x[e], q2);
                const uint32_t tv = shoup32(x[e2], w.w, w.wp, q);
                x[e] = u + tv;
                x[e2] = u + q2 - tv;
            } else {
                const uint32_t u = x[e], v = x[e2];
                if (fold_stage) {
                    x[e] = shoup32(u + v, fold.c.w, fold.c.wp, q);
                    x[e2] = shoup32(u + q2 - v, fold.cw.w, fold.cw.wp, q);
                } else {
                    x[e] = csub32(u + v, q2);
                    x[e2] = shoup32(u + q2 - v, w.w, w.wp, q);
                }
            }
        }
    }
}

template <int LOGS, int LINES, bool COLS, int LO, int HI, int E>
__device__ __forceinline__ void put32(uint32_t *lds, const uint32_t (&x)[E], int line, int t) {
#pragma unroll
    for (int e = 0; e < E; ++e) lds[Tile32<LOGS, LINES, COLS, E>::idx(line, k32<LO, HI, E>(t, e))] = x[e];
}
template <int LOGS, int LINES, bool COLS, int LO, int HI, int E>
__device__ __forceinline__ void get32(const uint32_t *lds, uint32_t (&x)[E], int line, int t) {
#pragma unroll
    for (int e = 0; e < E; ++e) x[e] = lds[Tile32<LOGS, LINES, COLS, E>::idx(line, k32<LO, HI, E>(t, e))];
}

// A whole pass in registers: forward enters in [HL, HH) and leaves in
// [LL, LH); inverse the other way round.  The caller synchronizes before the
// LDS tile is written again.
template <int LOGS, int LINES, bool COLS, bool FWD, int E, typename TW>
__device__ __forceinline__ void pass32(uint32_t (&x)[E], uint32_t *lds, int line, int t, uint32_t q, const TW &tws,
                                       const Last32 &fold) {
    using P = Ph32<LOGS, E>;
    constexpr bool FOLD = !FWD && COLS;
    if (FWD) {
        phase32<LOGS, true, false, P::HL, P::HH, E>(x, t, q, tws, fold);
        put32<LOGS, LINES, COLS, P::HL, P::HH, E>(lds, x, line, t);
        __syncthreads();
        get32<LOGS, LINES, COLS, P::ML, P::MH, E>(lds, x, line, t);
        phase32<LOGS, true, false, P::ML, P::MH, E>(x, t, q, tws, fold);
        if constexpr (P::THREE) {
            __syncthreads();
            put32<LOGS, LINES, COLS, P::ML, P::MH, E>(lds, x, line, t);
            __syncthreads();
            get32<LOGS, LINES, COLS, P::LL, P::LH, E>(lds, x, line, t);
            phase32<LOGS, true, false, P::LL, P::LH, E>(x, t, q, tws, fold);
        }
    } else {
        if constexpr (P::THREE) {
            phase32<LOGS, false, FOLD, P::LL, P::LH, E>(x, t, q, tws, fold);
            put32<LOGS, LINES, COLS, P::LL, P::LH, E>(lds, x, line, t);
            __syncthreads();
            get32<LOGS, LINES, COLS, P::ML, P::MH, E>(lds, x, line, t);
            __syncthreads();
        }
        phase32<LOGS, false, FOLD, P::ML, P::MH, E>(x, t, q, tws, fold);
        put32<LOGS, LINES, COLS, P::ML, P::MH, E>(lds, x, line, t);
        __syncthreads();
        get32<LOGS, LINES, COLS, P::HL, P::HH, E>(lds, x, line, t);
        phase32<LOGS, false, FOLD, P::HL, P::HH, E>(x, t, q, tws, fold);
    }
}

template <int LOGS, int LINES, bool COLS, int E = E32>
__device__ __forceinline__ void coords32(int tid, int &line, int &t) {
    if (COLS) {
        line = tid % LINES;
        t = tid / LINES;
    } else {
        t = tid % Tile32<LOGS, LINES, COLS, E>::T;
        line = tid / Tile32<LOGS, LINES, COLS, E>::T;
    }
}

// Load / store a thread's E32 elements of line lg in layout [LO, HI); a row
// pass in a [0, b) layout owns E32 consecutive words: four 16-byte accesses.
template <bool COLS, int LO, int HI, int E = E32>
__device__ __forceinline__ void load32(uint32_t (&x)[E], const uint32_t *__restrict__ src, int t, uint32_t lg,
                                       uint32_t n2) {
    if (!COLS && LO == 0) {
        const uint4 *p = reinterpret_cast<const uint4 *>(src + (lg << n2) + E * t);
#pragma unroll
        for (int c = 0; c < E / 4; ++c) {
            const uint4 v = p[c];
            x[4 * c] = v.x;
            x[4 * c + 1] = v.y;
            x[4 * c + 2] = v.z;
            x[4 * c + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = src[jdx32<COLS>(lg, k32<LO, HI, E>(t, e), n2)];
    }
}

template <bool COLS, int LO, int HI, int E = E32>
__device__ __forceinline__ void store32(const uint32_t (&x)[E], uint32_t *__restrict__ dst, int t, uint32_t lg,
                                        uint32_t n2) {
    if (!COLS && LO == 0) {
        uint4 *p = reinterpret_cast<uint4 *>(dst + (lg << n2) + E * t);
#pragma unroll
        for (int c = 0; c < E / 4; ++c) p[c] = make_uint4(x[4 * c], x[4 * c + 1], x[4 * c + 2], x[4 * c + 3]);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) dst[jdx32<COLS>(lg, k32<LO, HI, E>(t, e), n2)] = x[e];
    }
}

// ------------------------------------------------------------------ NTT passes

enum { P32_PLAIN = 0, P32_GATHER = 1, P32_REDUCE = 2, P32_EPI = 3 };

struct Pass32Args {
    const Shoup32 *tw;
    const Mod32 *mc;
    const Last32 *fold;     // inverse column pass: by cidx
    const Shoup32 *pinv;    // P32_EPI: P^-1 mod q_i, by cidx
    const uint32_t *in;
    uint32_t *out;
    size_t in_ys, out_ys;   // per blockIdx.y (polynomial) strides in words
    const uint32_t *uq;     // P32_EPI: u at uq + y uq_ys + cidx N
    size_t uq_ys;
    const uint32_t *b;      // P32_EPI: added to polynomial 1, gathered through gal[y / 2]
    uint32_t galois;        // P32_GATHER
    uint32_t *outs[HB32];   // P32_EPI: polynomial y at outs[y / 2] + (y % 2) out_ys
    uint32_t gal[HB32];
    uint32_t n, n1, n2;
    Map32 m;
};

template <int LOGS, int LINES, bool COLS, bool FWD, int IO>
__global__ void __launch_bounds__((Tile32<LOGS, LINES, COLS>::NT)) pass32_kernel(const Pass32Args a) {
    using TL = Tile32<LOGS, LINES, COLS>;
    using P = Ph32<LOGS>;
    constexpr int IN_LO = FWD ? P::HL : P::LL, IN_HI = FWD ? P::HH : P::LH;
    constexpr int OUT_LO = FWD ? P::LL : P::HL, OUT_HI = FWD ? P::LH : P::HH;
    __shared__ uint32_t lds[TL::WORDS];
    const uint32_t tiles = (1u << (COLS ? a.n2 : a.n1)) / LINES;
    const uint32_t li = blockIdx.x / tiles, tile = blockIdx.x % tiles, y = blockIdx.y;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = a.m.mod[li];
    const Mod32 mc = a.mc[mod];
    const uint32_t q = mc.q;
    const uint32_t *src = a.in + y * a.in_ys + (size_t)a.m.in_off[li] * N;
    uint32_t *dst = (IO == P32_EPI ? a.outs[y >> 1] + (y & 1) * a.out_ys : a.out + y * a.out_ys) +
                    (size_t)a.m.out_off[li] * N;
    int line, t;
    coords32<LOGS, LINES, COLS>(threadIdx.x, line, t);
    const uint32_t lg = tile * LINES + line;

    // ModDown epilogue operand u, issued before the pass input
    uint32_t uv[E32];
    if (IO == P32_EPI)
        load32<COLS, OUT_LO, OUT_HI>(uv, a.uq + y * a.uq_ys + (size_t)a.m.cidx[li] * N, t, lg, a.n2);
    uint32_t x[E32];
    if (IO == P32_GATHER) {
#pragma unroll
        for (int e = 0; e < E32; ++e) {
            const uint32_t j = jdx32<COLS>(lg, k32<IN_LO, IN_HI>(t, e), a.n2);
            x[e] = src[a.galois != 1 ? aut_eval_src(j, a.galois, a.n) : j];
        }
    } else {
        load32<COLS, IN_LO, IN_HI>(x, src, t, lg, a.n2);
    }
    const Last32 fold = (!FWD && COLS) ? a.fold[a.m.cidx[li]] : Last32{};
    if constexpr (COLS)
        pass32<LOGS, LINES, COLS, FWD>(x, lds, line, t, q, Tw32Cols{a.tw + (size_t)mod * N}, fold);
    else
        pass32<LOGS, LINES, COLS, FWD>(x, lds, line, t, q, Tw32Rows{a.tw + (size_t)mod * N, lg, a.n1}, fold);

    if (IO == P32_EPI) {
        const uint32_t ui = a.m.cidx[li];
        const uint32_t *bb = ((y & 1) && a.b) ? a.b + (size_t)ui * N : nullptr;
        const uint32_t g = a.gal[y >> 1];
        const Shoup32 pi = a.pinv[ui];
#pragma unroll
        for (int e = 0; e < E32; ++e) {
            const uint32_t j = jdx32<COLS>(lg, k32<OUT_LO, OUT_HI>(t, e), a.n2);
            const uint32_t z = csub32(csub32(x[e], 2 * q), q);
            uint32_t r = csub32(shoup32(uv[e] + q - z, pi.w, pi.wp, q), q);
            if (bb) r = csub32(r + bb[g != 1 ? aut_eval_src(j, g, a.n) : j], q);
            x[e] = r;
        }
    } else if (FWD && IO == P32_REDUCE) {
#pragma unroll
        for (int e = 0; e < E32; ++e) x[e] = csub32(csub32(x[e], 2 * q), q);
    } else if (!FWD && COLS) {
#pragma unroll
        for (int e = 0; e < E32; ++e) x[e] = csub32(x[e], q);  // canonical coefficients
    }
    store32<COLS, OUT_LO, OUT_HI>(x, dst, t, lg, a.n2);
}

template <bool COLS, bool FWD, int IO>
static hipError_t launch_pass32(const Ctx32 &c, const Pass32Args &a, uint32_t ys, hipStream_t s) {
    if (a.m.count == 0) return hipSuccess;
    constexpr int LINES = COLS ? COL32 : ROW32;
    const int logs = COLS ? (int)c.n1 : (int)c.n2;
    const uint32_t lines = 1u << (COLS ? c.n2 : c.n1);
    if (lines % LINES) return hipErrorInvalidValue;
    const dim3 grid(a.m.count * (lines / LINES), ys);
    switch (logs) {
#define P32_CASE(LG)                                                                                              \
    case LG:                                                                                                      \
        hipLaunchKernelGGL((pass32_kernel<LG, LINES, COLS, FWD, IO>), grid, dim3(Tile32<LG, LINES, COLS>::NT), 0, \
                           s, a);                                                                                 \
        break;
        P32_CASE(5)
        P32_CASE(6)
        P32_CASE(7)
        P32_CASE(8)
#undef P32_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static Pass32Args pass_args(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, bool fwd) {
    Pass32Args a{};
    a.tw = fwd ? c.tw_fwd : c.tw_inv;
    a.mc = c.mc;
    a.pinv = c.pinv;
    a.in = in;
    a.out = out;
    a.galois = 1;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.m = m;
    return a;
}

hipError_t launch32_fwd_cols(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, hipStream_t s,
                             uint32_t ys, size_t in_ys, size_t out_ys) {
    Pass32Args a = pass_args(c, m, in, out, true);
    a.in_ys = in_ys;
    a.out_ys = out_ys;
    return launch_pass32<true, true, P32_PLAIN>(c, a, ys, s);
}

hipError_t launch32_fwd_rows(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, hipStream_t s) {
    return launch_pass32<false, true, P32_REDUCE>(c, pass_args(c, m, in, out, true), 1, s);
}

hipError_t launch32_inv_rows(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, uint32_t galois,
                             hipStream_t s) {
    Pass32Args a = pass_args(c, m, in, out, false);
    a.galois = galois;
    return galois != 1 ? launch_pass32<false, false, P32_GATHER>(c, a, 1, s)
                       : launch_pass32<false, false, P32_PLAIN>(c, a, 1, s);
}

hipError_t launch32_inv_cols(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, const Last32 *fold,
                             hipStream_t s, uint32_t ys, size_t in_ys, size_t out_ys) {
    Pass32Args a = pass_args(c, m, in, out, false);
    a.fold = fold;
    a.in_ys = in_ys;
    a.out_ys = out_ys;
    return launch_pass32<true, false, P32_PLAIN>(c, a, ys, s);
}

hipError_t launch32_rows_epi(const Ctx32 &c, uint32_t level, const uint32_t *z, const uint32_t *uq,
                             const uint32_t *b, uint32_t nrot, uint32_t *const *outs, const uint32_t *gals,
                             hipStream_t s) {
    if (nrot == 0 || nrot > HB32) return hipErrorInvalidValue;
    Map32 m{};
    m.count = level;
    for (uint32_t i = 0; i < level; ++i) {
        m.in_off[i] = (uint16_t)i;
        m.out_off[i] = (uint16_t)i;
        m.mod[i] = (uint8_t)i;
        m.cidx[i] = (uint16_t)i;
    }
    Pass32Args a = pass_args(c, m, z, nullptr, true);
    const size_t pl = (size_t)level * c.n;
    a.in_ys = (size_t)c.L * c.n;
    a.out_ys = pl;
    a.uq = uq;
    a.uq_ys = pl;
    a.b = b;
    for (uint32_t r = 0; r < nrot; ++r) {
        a.outs[r] = outs[r];
        a.gal[r] = gals[r];
    }
    return launch_pass32<false, true, P32_EPI>(c, a, 2 * nrot, s);
}

// ------------------------------------------------------------------ NewLimb

struct Conv32Args {
    const uint32_t *in;
    uint32_t *out;
    const uint32_t *conv;
    const Mod32 *mc;
    uint32_t n, level, L, K, alpha, tgroups;
};

// One thread = one coefficient and one group of target limbs: its source
// residues are loaded once and the group's targets are produced from them
// (64-bit exact sums, one reduction).  blockIdx.z picks the group (targets
// [z T, (z+1) T) of the nt, T = ceil(nt / tgroups)), so that a launch has
// several blocks per CU; the groups re-read the sources from L2.
//   MODUP:   digit j = blockIdx.y, sources y[j alpha ..), targets t of
//            Q_level U P outside the digit -> out[(j E + t) N], row j E + t;
//   ModDown: polynomial p = blockIdx.y, sources the K P limbs at in + p K N,
//            targets the level q limbs -> out + p L N, row i.
template <bool MODUP, int MAXS>
__global__ void __launch_bounds__(256) conv32_kernel(const Conv32Args a) {
    constexpr int MAXT = 256;
    __shared__ uint32_t kc[MAXT * MAXS];
    __shared__ Mod32 mt[MAXT];
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t j = blockIdx.y;
    const uint32_t lo = MODUP ? j * a.alpha : 0;
    const uint32_t ns = MODUP ? min(a.alpha, a.level - lo) : a.K;
    const uint32_t E = a.level + a.K;
    const uint32_t nt = MODUP ? E : a.level;
    const uint32_t cstride = MODUP ? a.alpha : a.K;
    const uint32_t *rows = a.conv + (size_t)(MODUP ? j * E : 0) * cstride;
    for (uint32_t i = threadIdx.x; i < nt * MAXS; i += blockDim.x) {
        const uint32_t tt = i / MAXS, ss = i % MAXS;
        kc[i] = (ss < ns) ? rows[(size_t)tt * cstride + ss] : 0;
    }
    for (uint32_t tt = threadIdx.x; tt < nt; tt += blockDim.x) {
        const uint32_t mod = MODUP ? (tt < a.level ? tt : a.L + (tt - a.level)) : tt;
        mt[tt] = a.mc[mod];
    }
    const uint32_t *src = MODUP ? a.in + (size_t)lo * N + c : a.in + (size_t)j * a.K * N + c;
    uint32_t y[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) y[i] = (i < (int)ns) ? src[(size_t)i * N] : 0;
    __syncthreads();
    uint32_t *dst = MODUP ? a.out + c : a.out + (size_t)j * a.L * N + c;
    const uint32_t per = (nt + a.tgroups - 1) / a.tgroups;
    const uint32_t t0 = blockIdx.z * per, t1 = min(nt, t0 + per);
    for (uint32_t tt = t0; tt < t1; ++tt) {
        if (MODUP && tt >= lo && tt < lo + ns) continue;
        const uint32_t *kr = kc + tt * MAXS;
        uint64_t acc = 0;
#pragma unroll
        for (int i = 0; i < MAXS; ++i) acc += (uint64_t)y[i] * kr[i];
        dst[(size_t)(MODUP ? j * E + tt : tt) * N] = reduce64_32(acc, mt[tt]);
    }
}

template <bool MODUP>
static hipError_t launch_conv32_t(const Conv32Args &a, uint32_t ns, dim3 grid, hipStream_t s) {
    if (ns <= 8) hipLaunchKernelGGL((conv32_kernel<MODUP, 8>), grid, dim3(256), 0, s, a);
    else if (ns <= 16) hipLaunchKernelGGL((conv32_kernel<MODUP, 16>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// target groups per launch: about 8 targets per thread, at least one group
static uint32_t conv_groups(uint32_t nt) { return std::max<uint32_t>(1, nt / 8); }

hipError_t launch32_conv_modup(const Ctx32 &c, const uint32_t *y, uint32_t level, uint32_t *ext, hipStream_t s) {
    if (level + c.K > 256) return hipErrorInvalidValue;
    const uint32_t g = conv_groups(level + c.K);
    Conv32Args a{y, ext, c.conv_modup + c.conv_modup_off[level], c.mc, c.log_n, level, c.L, c.K, c.alpha, g};
    const uint32_t beta = (level + c.alpha - 1) / c.alpha;
    return launch_conv32_t<true>(a, c.alpha, dim3((c.n + 255) / 256, beta, g), s);
}

hipError_t launch32_conv_moddown(const Ctx32 &c, const uint32_t *pc, uint32_t level, uint32_t polys, uint32_t *z,
                                 hipStream_t s) {
    const uint32_t g = conv_groups(level);
    Conv32Args a{pc, z, c.conv_moddown, c.mc, c.log_n, level, c.L, c.K, c.alpha, g};
    return launch_conv32_t<false>(a, c.K, dim3((c.n + 255) / 256, polys, g), s);
}

// ------------------------------------------------------------------ KSKInnerProd

struct Ksk32Args {
    const uint32_t *ext;   // [beta][E][N] new limbs after the forward column pass
    const uint32_t *a;     // input a, [level][N] evaluation form (the digits' own limbs)
    const uint32_t *ksk;   // [dnum][2][L+K][N]
    uint32_t *uq, *pc;
    const Shoup32 *twf, *twi;
    const Mod32 *mc;
    uint32_t galois, n, n1, n2, level, L, K, E, alpha, beta;
    uint32_t direct;  // ext holds the new limbs fully transformed: gather them too
};

// One block = one limb t of Q_level U P and ROW32 rows (the special-prime
// limbs first): for each digit, the limb's forward row pass (or the digit's
// own limb gathered from a through the automorphism), reduced to [0, q),
// times the key rows, summed exactly in 64 bits (folded every 16 digits).
// With `direct` (hoisted rotations) the new limbs are already in evaluation
// form and are gathered through the automorphism like the own limbs.
// q limbs store u, v; P limbs run ModDown's inverse row pass first.
template <int LOGS, int E>
__global__ void __launch_bounds__((Tile32<LOGS, ROW32, false, E>::NT)) ksk32_kernel(const Ksk32Args a) {
    using TL = Tile32<LOGS, ROW32, false, E>;
    using P = Ph32<LOGS, E>;
    __shared__ uint32_t lds[TL::WORDS];
    const uint32_t tiles = (1u << a.n1) / ROW32;
    const uint32_t tgt = (blockIdx.x / tiles + a.level) % a.E;
    const uint32_t tile = blockIdx.x % tiles;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = tgt < a.level ? tgt : a.L + (tgt - a.level);
    const Mod32 mc = a.mc[mod];
    const uint32_t q = mc.q;
    const size_t KL = (size_t)a.L + a.K;
    const uint32_t own = tgt < a.level ? tgt / a.alpha : 0xffffffffu;
    int line, t;
    coords32<LOGS, ROW32, false, E>(threadIdx.x, line, t);
    const uint32_t lg = tile * ROW32 + line;
    const uint32_t slot0 = (lg << a.n2) + E * t;  // forward output layout: E consecutive slots

    uint64_t ua[E], va[E];
#pragma unroll
    for (int e = 0; e < E; ++e) ua[e] = va[e] = 0;
    bool lds_used = false;
    for (uint32_t jd = 0; jd < a.beta; ++jd) {
        if (jd && (jd & 15) == 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                ua[e] = reduce64_32(ua[e], mc);
                va[e] = reduce64_32(va[e], mc);
            }
        }
        uint32_t xv[E];
        if (jd == own || a.direct) {
            const uint32_t *src = jd == own ? a.a + (size_t)tgt * N : a.ext + ((size_t)jd * a.E + tgt) * N;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t j = slot0 + e;
                xv[e] = src[a.galois != 1 ? aut_eval_src(j, a.galois, a.n) : j];
            }
        } else {
            const uint32_t *src = a.ext + ((size_t)jd * a.E + tgt) * N;
            load32<false, P::HL, P::HH, E>(xv, src, t, lg, a.n2);
            if (lds_used) __syncthreads();
            pass32<LOGS, ROW32, false, true>(xv, lds, line, t, q, Tw32Rows{a.twf + (size_t)mod * N, lg, a.n1},
                                             Last32{});
            lds_used = true;
#pragma unroll
            for (int e = 0; e < E; ++e) xv[e] = csub32(csub32(xv[e], 2 * q), q);
        }
        const uint4 *k0 = reinterpret_cast<const uint4 *>(a.ksk + ((size_t)(2 * jd) * KL + mod) * N + slot0);
        const uint4 *k1 = reinterpret_cast<const uint4 *>(a.ksk + ((size_t)(2 * jd + 1) * KL + mod) * N + slot0);
#pragma unroll
        for (int c4 = 0; c4 < E / 4; ++c4) {
            const uint4 p0 = k0[c4], p1 = k1[c4];
            const uint32_t kv0[4] = {p0.x, p0.y, p0.z, p0.w}, kv1[4] = {p1.x, p1.y, p1.z, p1.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ua[4 * c4 + i] += (uint64_t)xv[4 * c4 + i] * kv0[i];
                va[4 * c4 + i] += (uint64_t)xv[4 * c4 + i] * kv1[i];
            }
        }
    }
    uint32_t u[E], v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        u[e] = reduce64_32(ua[e], mc);
        v[e] = reduce64_32(va[e], mc);
    }
    if (tgt < a.level) {
        uint4 *du = reinterpret_cast<uint4 *>(a.uq + (size_t)tgt * N + slot0);
        uint4 *dv = reinterpret_cast<uint4 *>(a.uq + ((size_t)a.level + tgt) * N + slot0);
#pragma unroll
        for (int c4 = 0; c4 < E / 4; ++c4) {
            du[c4] = make_uint4(u[4 * c4], u[4 * c4 + 1], u[4 * c4 + 2], u[4 * c4 + 3]);
            dv[c4] = make_uint4(v[4 * c4], v[4 * c4 + 1], v[4 * c4 + 2], v[4 * c4 + 3]);
        }
        return;
    }
    const uint32_t kp = tgt - a.level;
    const Tw32Rows twi{a.twi + (size_t)mod * N, lg, a.n1};
    if (lds_used) __syncthreads();
    pass32<LOGS, ROW32, false, false>(u, lds, line, t, q, twi, Last32{});
#pragma unroll
    for (int e = 0; e < E; ++e) a.pc[(size_t)kp * N + jdx32<false>(lg, k32<P::HL, P::HH, E>(t, e), a.n2)] = u[e];
    __syncthreads();
    pass32<LOGS, ROW32, false, false>(v, lds, line, t, q, twi, Last32{});
#pragma unroll
    for (int e = 0; e < E; ++e)
        a.pc[((size_t)a.K + kp) * N + jdx32<false>(lg, k32<P::HL, P::HH, E>(t, e), a.n2)] = v[e];
}

hipError_t launch32_ksk(const Ctx32 &c, const uint32_t *ext, bool direct, const uint32_t *a, uint32_t galois,
                        uint32_t level, const uint32_t *ksk, uint32_t *uq, uint32_t *pc, hipStream_t s) {
    Ksk32Args k{};
    k.ext = ext;
    k.direct = direct ? 1 : 0;
    k.a = a;
    k.ksk = ksk;
    k.uq = uq;
    k.pc = pc;
    k.twf = c.tw_fwd;
    k.twi = c.tw_inv;
    k.mc = c.mc;
    k.galois = galois;
    k.n = c.log_n;
    k.n1 = c.n1;
    k.n2 = c.n2;
    k.level = level;
    k.L = c.L;
    k.K = c.K;
    k.E = level + c.K;
    k.alpha = c.alpha;
    k.beta = (level + c.alpha - 1) / c.alpha;
    const uint32_t lines = 1u << c.n1;
    if (lines % ROW32) return hipErrorInvalidValue;
    const dim3 grid(k.E * (lines / ROW32));
    constexpr int E = EK32;
    switch (c.n2) {
        case 5: hipLaunchKernelGGL((ksk32_kernel<5, E>), grid, dim3(Tile32<5, ROW32, false, E>::NT), 0, s, k); break;
        case 6: hipLaunchKernelGGL((ksk32_kernel<6, E>), grid, dim3(Tile32<6, ROW32, false, E>::NT), 0, s, k); break;
        case 7: hipLaunchKernelGGL((ksk32_kernel<7, E>), grid, dim3(Tile32<7, ROW32, false, E>::NT), 0, s, k); break;
        case 8: hipLaunchKernelGGL((ksk32_kernel<8, E>), grid, dim3(Tile32<8, ROW32, false, E>::NT), 0, s, k); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace w32
}  // namespace hks
