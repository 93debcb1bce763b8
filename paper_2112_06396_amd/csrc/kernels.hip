// HIP kernels for gfx950: negacyclic NTT / iNTT (Sec. 2.3), fast basis
// conversion (NewLimb of Algorithm "ModUp", also used by ModDown),
// KSKInnerProd, ModDown's final step, Automorph and the elementwise steps of
// PtMult / Mult (Algorithms 1-2) and Rescale.
//
// NTT structure.  N = 2^n is viewed as a 2^n1 x 2^n2 matrix (row r, column
// c, element j = r*2^n2 + c).  The forward transform is the merged
// Cooley-Tukey negacyclic NTT with bit-reversed output: stage s (s = 0..n-1)
// pairs j and j + N/2^(s+1) with twiddle psi^brv(2^s + (j >> (n-s))).  Stages
// 0..n1-1 only combine elements of one column ("column pass"), stages
// n1..n-1 only elements of one row ("row pass").  The inverse runs the
// Gentleman-Sande butterflies in the reverse order (row pass first), with
// N^-1 and any per-limb scale folded into the last stage.
//
// Each pass kernel loads a tile of LINES lines into LDS with coalesced
// accesses, then runs phases of up to four stages: every thread holds 16
// elements in registers, does up to 32 butterflies, and exchanges through
// LDS between phases.  Values stay lazy (not fully reduced) between stages:
// forward outputs grow by < 2q per stage (< 35q < 2^56 after 16 stages),
// inverse values stay in [0, 2q).
#include <hip/hip_runtime.h>

#include "hks_internal.h"
#include "modarith.h"

namespace hks {

// ------------------------------------------------------------------ timing

static hipEvent_t prof_event(const Ctx &c) {
    if (!c.prof_pool.empty()) {
        hipEvent_t e = c.prof_pool.back();
        c.prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(const Ctx &ctx, int k, hipStream_t st) : c(ctx), cls(k), s(st), on(false) {
    if (!((c.prof_mask >> cls) & 1u)) return;
    hipEvent_t a = prof_event(c), b = prof_event(c);
    if (!a || !b) return;
    if (hipEventRecord(a, s) != hipSuccess) return;
    c.prof_ev[cls].push_back({a, b});
    on = true;
}

ProfScope::~ProfScope() {
    if (on) (void)hipEventRecord(c.prof_ev[cls].back().second, s);
}

void prof_reset(const Ctx &c) {
    for (int k = 0; k < HKS_K_COUNT; ++k) {
        for (auto &p : c.prof_ev[k]) {
            c.prof_pool.push_back(p.first);
            c.prof_pool.push_back(p.second);
        }
        c.prof_ev[k].clear();
    }
}

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ uint32_t brev_n(uint32_t x, uint32_t n) { return __brev(x) >> (32 - n); }

// Source slot of output slot j under X -> X^g in the bit-reversed evaluation
// order: slot j holds a(psi^(2 brv(j) + 1)); psi^((2 brv(j)+1) g) is held by
// slot brv(((2 brv(j) + 1) g mod 2N - 1) / 2).
__device__ __forceinline__ uint32_t aut_eval_src(uint32_t j, uint32_t g, uint32_t n) {
    uint32_t k = brev_n(j, n);
    uint32_t odd = ((2u * k + 1u) * g) & ((2u << n) - 1u);
    return brev_n((odd - 1u) >> 1, n);
}

template <int LOGS, int LINES, bool COLS>
struct Tile {
    static constexpr int S = 1 << LOGS;
    static constexpr int T = S / 16;         // threads per line
    static constexpr int NT = LINES * T;     // threads per block
    static constexpr int ROWP = S + S / 16;  // padded row length (row tiles)
    static constexpr int COLP = LINES + 1;   // padded k-row length (column tiles)
    static constexpr int WORDS = COLS ? S * COLP : LINES * ROWP;
    __device__ static __forceinline__ int idx(int line, int k) {
        return COLS ? k * COLP + line : line * ROWP + k + (k >> 4);
    }
};

// One phase: bits [LO, HI) of the sub-index k, 16 elements per thread.
// FWD: Cooley-Tukey stages from bit HI-1 down to LO.  !FWD: Gentleman-Sande
// stages from bit LO up to HI-1; the global stage 0 (only reached by the
// inverse column pass) uses the folded constants `fold`.
template <int LOGS, int LINES, bool COLS, bool FWD, int LO, int HI>
__device__ __forceinline__ void ntt_phase(uint64_t *lds, int line, int t, uint32_t line_g,
                                          int sigma0, int n, int n2, uint64_t q,
                                          const Shoup *__restrict__ tw, const LastInv &fold) {
    using TL = Tile<LOGS, LINES, COLS>;
    constexpr int B = HI - LO;
    constexpr int G = 16 >> B;
    uint64_t x[16];
    int kk[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        int v = e & ((1 << B) - 1), g = e >> B;
        int r = t * G + g;
        int k = ((r >> LO) << HI) | (v << LO) | (r & ((1 << LO) - 1));
        kk[e] = k;
        x[e] = lds[TL::idx(line, k)];
    }
    const uint64_t q2 = 2 * q;
#pragma unroll
    for (int st = 0; st < B; ++st) {
        const int bit = FWD ? (HI - 1 - st) : (LO + st);
        const int vb = bit - LO;
        const int sigma = (COLS ? 0 : sigma0) + LOGS - 1 - bit;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if ((e >> vb) & 1) continue;
            const int e2 = e + (1 << vb);
            const uint32_t k = (uint32_t)kk[e];
            const uint32_t j = COLS ? (k << n2) : ((line_g << n2) | k);
            if (FWD) {
                const Shoup w = tw[(1u << sigma) + (j >> (n - sigma))];
                const uint64_t u = x[e];
                const uint64_t tv = mul_shoup_lazy(x[e2], w.w, w.wp, q);
                x[e] = u + tv;
                x[e2] = u + q2 - tv;
            } else {
                const uint64_t u = x[e], v = x[e2];
                if (COLS && sigma == 0) {
                    x[e] = mul_shoup(u + v, fold.c.w, fold.c.wp, q);
                    x[e2] = mul_shoup(u + q2 - v, fold.cw.w, fold.cw.wp, q);
                } else {
                    const Shoup w = tw[(1u << sigma) + (j >> (n - sigma))];
                    x[e] = csub(u + v, q2);
                    x[e2] = mul_shoup_lazy(u + q2 - v, w.w, w.wp, q);
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[TL::idx(line, kk[e])] = x[e];
}

template <int LOGS, int LINES, bool COLS, bool FWD>
__device__ __forceinline__ void ntt_all_phases(uint64_t *lds, int line, int t, uint32_t line_g,
                                               int sigma0, int n, int n2, uint64_t q,
                                               const Shoup *__restrict__ tw, const LastInv &fold) {
    // phases of four bits from the top: [LOGS-4, LOGS), [LOGS-8, LOGS-4), ...
    constexpr int P0L = LOGS - 4;
    constexpr int P1H = P0L, P1L = (P0L - 4) > 0 ? (P0L - 4) : 0;
    constexpr int P2H = P1L, P2L = 0;
    static_assert(LOGS >= 5 && LOGS <= 12, "sub-transform size");
    if (FWD) {
        ntt_phase<LOGS, LINES, COLS, true, P0L, LOGS>(lds, line, t, line_g, sigma0, n, n2, q, tw, fold);
        __syncthreads();
        ntt_phase<LOGS, LINES, COLS, true, P1L, P1H>(lds, line, t, line_g, sigma0, n, n2, q, tw, fold);
        if constexpr (P2H > P2L) {
            __syncthreads();
            ntt_phase<LOGS, LINES, COLS, true, P2L, P2H>(lds, line, t, line_g, sigma0, n, n2, q, tw, fold);
        }
    } else {
        if constexpr (P2H > P2L) {
            ntt_phase<LOGS, LINES, COLS, false, P2L, P2H>(lds, line, t, line_g, sigma0, n, n2, q, tw, fold);
            __syncthreads();
        }
        ntt_phase<LOGS, LINES, COLS, false, P1L, P1H>(lds, line, t, line_g, sigma0, n, n2, q, tw, fold);
        __syncthreads();
        ntt_phase<LOGS, LINES, COLS, false, P0L, LOGS>(lds, line, t, line_g, sigma0, n, n2, q, tw, fold);
    }
}

struct NttArgs {
    const Ctx *ctx;  // host-side only (timing); not read by kernels
    const uint64_t *in;
    uint64_t *out;
    const Shoup *tw;       // [M][N] forward or inverse table
    const ModC *mc;
    const LastInv *li;     // folded last inverse stage, indexed by cidx
    size_t in_bstride, out_bstride;
    uint32_t n, n1, n2, galois;
    LimbMap m;
};

enum { IO_PLAIN = 0, IO_GATHER = 1, IO_REDUCE = 2 };

// One pass over tiles of LINES lines.  COLS: lines are columns (sub-transform
// over rows, stride 2^n2), sigma0 = 0, LOGS = n1.  !COLS: lines are rows
// (contiguous), sigma0 = n1, LOGS = n2.
template <int LOGS, int LINES, bool COLS, bool FWD, int IO>
__global__ void __launch_bounds__((Tile<LOGS, LINES, COLS>::NT))
ntt_pass_kernel(const NttArgs a) {
    using TL = Tile<LOGS, LINES, COLS>;
    __shared__ uint64_t lds[TL::WORDS];
    const uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
    const uint32_t tiles = lines_per_limb / LINES;
    const uint32_t li = blockIdx.x / tiles;
    const uint32_t tile = blockIdx.x % tiles;
    const uint32_t b = blockIdx.y;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = a.m.mod[li];
    const uint64_t q = a.mc[mod].q;
    const uint64_t *src = a.in + b * a.in_bstride + (size_t)a.m.in_off[li] * N;
    uint64_t *dst = a.out + b * a.out_bstride + (size_t)a.m.out_off[li] * N;
    const Shoup *tw = a.tw + (size_t)mod * N;
    const int tid = threadIdx.x;
    const uint32_t line0 = tile * LINES;

    // coalesced load of the tile
#pragma unroll 4
    for (int e = tid; e < LINES * TL::S; e += TL::NT) {
        int line, k;
        uint32_t j;
        if (COLS) {
            k = e / LINES;
            line = e % LINES;
            j = ((uint32_t)k << a.n2) + line0 + line;
        } else {
            line = e / TL::S;
            k = e % TL::S;
            j = ((line0 + line) << a.n2) + k;
        }
        uint32_t sj = (IO == IO_GATHER) ? aut_eval_src(j, a.galois, a.n) : j;
        lds[TL::idx(line, k)] = src[sj];
    }
    __syncthreads();

    int line, t;
    if (COLS) {
        line = tid % LINES;
        t = tid / LINES;
    } else {
        t = tid % TL::T;
        line = tid / TL::T;
    }
    const LastInv fold = (!FWD && COLS) ? a.li[a.m.cidx[li]] : LastInv{};
    ntt_all_phases<LOGS, LINES, COLS, FWD>(lds, line, t, line0 + line, COLS ? 0 : (int)a.n1, (int)a.n,
                                           (int)a.n2, q, tw, fold);
    __syncthreads();

    const uint64_t mu = a.mc[mod].mu;
#pragma unroll 4
    for (int e = tid; e < LINES * TL::S; e += TL::NT) {
        int ln, k;
        uint32_t j;
        if (COLS) {
            k = e / LINES;
            ln = e % LINES;
            j = ((uint32_t)k << a.n2) + line0 + ln;
        } else {
            ln = e / TL::S;
            k = e % TL::S;
            j = ((line0 + ln) << a.n2) + k;
        }
        uint64_t v = lds[TL::idx(ln, k)];
        if (IO == IO_REDUCE) v = reduce64(v, q, mu);
        dst[j] = v;
    }
}

template <int LOGS, int LINES, bool COLS, bool FWD, int IO>
static hipError_t launch_pass(const NttArgs &a, uint32_t count, uint32_t batch, hipStream_t s) {
    using TL = Tile<LOGS, LINES, COLS>;
    ProfScope ps(*a.ctx, FWD ? (COLS ? HKS_K_NTT_FWD_COLS : HKS_K_NTT_FWD_ROWS)
                             : (COLS ? HKS_K_NTT_INV_COLS : HKS_K_NTT_INV_ROWS), s);
    uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
    dim3 grid(count * (lines_per_limb / LINES), batch);
    hipLaunchKernelGGL((ntt_pass_kernel<LOGS, LINES, COLS, FWD, IO>), grid, dim3(TL::NT), 0, s, a);
    return hipGetLastError();
}

template <bool COLS, bool FWD, int IO>
static hipError_t dispatch_pass(const NttArgs &a, int logs, uint32_t count, uint32_t batch, hipStream_t s) {
    switch (logs) {
        case 5: return launch_pass<5, 16, COLS, FWD, IO>(a, count, batch, s);
        case 6: return launch_pass<6, 16, COLS, FWD, IO>(a, count, batch, s);
        case 7: return launch_pass<7, 16, COLS, FWD, IO>(a, count, batch, s);
        case 8: return launch_pass<8, 16, COLS, FWD, IO>(a, count, batch, s);
        default: return hipErrorInvalidValue;
    }
}

static void limb_chunk(const LimbMap &src, uint32_t first, uint32_t cnt, LimbMap &dst) {
    dst.count = cnt;
    for (uint32_t i = 0; i < cnt; ++i) {
        dst.in_off[i] = src.in_off[first + i];
        dst.out_off[i] = src.out_off[first + i];
        dst.mod[i] = src.mod[first + i];
        dst.cidx[i] = src.cidx[first + i];
    }
}

hipError_t launch_ntt_fwd(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                          uint32_t batch, size_t in_bstride, size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a{};
    a.ctx = &c;
    a.tw = c.tw_fwd;
    a.mc = c.mc;
    a.li = c.li_plain;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.galois = 1;
    a.m = m;
    // pass 1 (columns): in -> out
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    hipError_t e = dispatch_pass<true, true, IO_PLAIN>(a, c.n1, m.count, batch, s);
    if (e != hipSuccess) return e;
    // pass 2 (rows): out -> out
    a.in = out;
    a.in_bstride = out_bstride;
    for (uint32_t i = 0; i < m.count; ++i) a.m.in_off[i] = m.out_off[i];
    return dispatch_pass<false, true, IO_REDUCE>(a, c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                          const LastInv *li, uint32_t galois, uint32_t batch, size_t in_bstride,
                          size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a{};
    a.ctx = &c;
    a.tw = c.tw_inv;
    a.mc = c.mc;
    a.li = li;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.galois = galois;
    a.m = m;
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    // pass 1 (rows), optional automorph gather
    hipError_t e = (galois != 1) ? dispatch_pass<false, false, IO_GATHER>(a, c.n2, m.count, batch, s)
                                 : dispatch_pass<false, false, IO_PLAIN>(a, c.n2, m.count, batch, s);
    if (e != hipSuccess) return e;
    a.in = out;
    a.in_bstride = out_bstride;
    a.galois = 1;
    for (uint32_t i = 0; i < m.count; ++i) a.m.in_off[i] = m.out_off[i];
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

// ------------------------------------------------------------------ basis conversion

struct ConvArgs {
    const uint64_t *in;
    uint64_t *out;
    const uint64_t *conv;  // [n_src][stride]
    const ModC *mc;
    size_t in_bstride, out_bstride;
    uint32_t N, n_src, stride;
    LimbMap m;  // out_off, mod, cidx (= column of the conversion table)
};

// out_t = sum_i in_i * conv[i][t] mod m_t, one coefficient per thread, 128-bit
// lazy accumulation and one Barrett reduction per output (Sec. 2.2).
template <int MAXS>
__global__ void __launch_bounds__(256) conv_kernel(const ConvArgs a) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.N) return;
    const uint32_t b = blockIdx.y;
    const uint64_t *src = a.in + b * a.in_bstride + c;
    uint64_t y[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) y[i] = (i < (int)a.n_src) ? src[(size_t)i * a.N] : 0;
    uint64_t *dst = a.out + b * a.out_bstride + c;
    for (uint32_t o = 0; o < a.m.count; ++o) {
        const uint32_t col = a.m.cidx[o];
        const ModC mcv = a.mc[a.m.mod[o]];
        Acc128 acc;
#pragma unroll
        for (int i = 0; i < MAXS; ++i)
            if (i < (int)a.n_src) acc.mac(y[i], a.conv[(size_t)i * a.stride + col]);
        dst[(size_t)a.m.out_off[o] * a.N] = acc.reduce(mcv.q, mcv.mu);
    }
}

hipError_t launch_conv_map(const Ctx &c, const uint64_t *in, uint32_t n_src, const uint64_t *conv,
                           uint32_t stride, uint64_t *out, const LimbMap &m, uint32_t batch,
                           size_t in_bstride, size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    ConvArgs a{};
    a.in = in;
    a.out = out;
    a.conv = conv;
    a.mc = c.mc;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    a.N = c.n;
    a.n_src = n_src;
    a.stride = stride;
    a.m = m;
    dim3 grid((c.n + 255) / 256, batch);
    ProfScope ps(c, HKS_K_CONV, s);
    if (n_src <= 4) hipLaunchKernelGGL(conv_kernel<4>, grid, dim3(256), 0, s, a);
    else if (n_src <= 8) hipLaunchKernelGGL(conv_kernel<8>, grid, dim3(256), 0, s, a);
    else if (n_src <= 12) hipLaunchKernelGGL(conv_kernel<12>, grid, dim3(256), 0, s, a);
    else if (n_src <= 16) hipLaunchKernelGGL(conv_kernel<16>, grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------ automorph

struct AutArgs {
    const uint64_t *in;
    uint64_t *out;
    const ModC *mc;
    size_t in_bstride, out_bstride;
    uint32_t n, galois, ginv;
    LimbMap m;
};

template <bool EVAL>
__global__ void __launch_bounds__(256) automorph_kernel(const AutArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t li = blockIdx.z;
    const uint32_t b = blockIdx.y;
    if (j >= N) return;
    const uint64_t *src = a.in + b * a.in_bstride + (size_t)a.m.in_off[li] * N;
    uint64_t *dst = a.out + b * a.out_bstride + (size_t)a.m.out_off[li] * N;
    if (EVAL) {
        dst[j] = src[aut_eval_src(j, a.galois, a.n)];
    } else {
        // y(X) = x(X^g): output coefficient j comes from i = j * g^-1 mod 2N,
        // negated when i >= N (X^N = -1).
        const uint32_t i = (j * a.ginv) & ((2u << a.n) - 1u);
        const uint64_t q = a.mc[a.m.mod[li]].q;
        if (i < N) {
            dst[j] = src[i];
        } else {
            uint64_t v = src[i - N];
            dst[j] = v ? q - v : 0;
        }
    }
}

hipError_t launch_automorph(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                            uint32_t galois, int eval_domain, uint32_t batch, size_t in_bstride,
                            size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    AutArgs a{};
    a.in = in;
    a.out = out;
    a.mc = c.mc;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    a.n = c.log_n;
    a.galois = galois;
    uint32_t two_n = 2u * c.n;
    a.ginv = (uint32_t)h_powmod(galois, (two_n / 2) - 1, two_n);  // g^(N-1) = g^-1 in (Z/2N)^*
    a.m = m;
    dim3 grid((c.n + 255) / 256, batch, m.count);
    ProfScope ps(c, HKS_K_AUTOMORPH, s);
    if (eval_domain) hipLaunchKernelGGL(automorph_kernel<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(automorph_kernel<false>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ KSKInnerProd

struct KskArgs {
    const uint64_t *ext;  // [beta][E][N]
    const uint64_t *ksk;  // [dnum][2][L+K][N]
    uint64_t *uv;         // [2][E][N]
    const ModC *mc;
    size_t ext_bstride, uv_bstride;
    uint32_t n, level, L, K, E, beta, galois;
};

// u_t = sum_j ext_j,t * ksk[j][0][kappa(t)], v_t likewise with row 1; the
// optional automorph (HRotate) gathers ext slots.  128-bit lazy sums.
__global__ void __launch_bounds__(256) ksk_kernel(const KskArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t t = blockIdx.z;
    const uint32_t b = blockIdx.y;
    if (c >= N) return;
    const uint32_t mod = t < a.level ? t : a.L + (t - a.level);
    const uint32_t kt = mod;  // key limb index equals the modulus index
    const ModC mcv = a.mc[mod];
    const uint32_t sc = (a.galois != 1) ? aut_eval_src(c, a.galois, a.n) : c;
    const size_t KL = (size_t)a.L + a.K;
    const uint64_t *ext = a.ext + b * a.ext_bstride + (size_t)t * N + sc;
    Acc128 u, v;
    for (uint32_t j = 0; j < a.beta; ++j) {
        uint64_t x = ext[(size_t)j * a.E * N];
        const uint64_t *k0 = a.ksk + ((size_t)(2 * j) * KL + kt) * N + c;
        u.mac(x, k0[0]);
        v.mac(x, k0[KL * N]);
    }
    uint64_t *uv = a.uv + b * a.uv_bstride + (size_t)t * N + c;
    uv[0] = u.reduce(mcv.q, mcv.mu);
    uv[(size_t)a.E * N] = v.reduce(mcv.q, mcv.mu);
}

hipError_t launch_ksk(const Ctx &c, const uint64_t *ext, uint32_t level, uint32_t beta,
                      const uint64_t *ksk, uint64_t *uv, uint32_t galois, uint32_t batch,
                      size_t ext_bstride, size_t uv_bstride, hipStream_t s) {
    KskArgs a{};
    a.ext = ext;
    a.ksk = ksk;
    a.uv = uv;
    a.mc = c.mc;
    a.ext_bstride = ext_bstride;
    a.uv_bstride = uv_bstride;
    a.n = c.log_n;
    a.level = level;
    a.L = c.L;
    a.K = c.K;
    a.E = level + c.K;
    a.beta = beta;
    a.galois = galois;
    dim3 grid((c.n + 255) / 256, batch, a.E);
    ProfScope ps(c, HKS_K_KSK, s);
    hipLaunchKernelGGL(ksk_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ ModDown final step

struct MdEpiArgs {
    const uint64_t *x, *z, *add;
    uint64_t *out;
    const ModC *mc;
    const Shoup *pinv;
    size_t x_bstride, z_bstride, out_bstride, add_pstride;
    uint32_t n, add_galois, add_mask;
};

__global__ void __launch_bounds__(256) moddown_epi_kernel(const MdEpiArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t i = blockIdx.z;
    const uint32_t b = blockIdx.y;
    if (c >= N) return;
    const uint64_t q = a.mc[i].q;
    const Shoup pi = a.pinv[i];
    const size_t off = (size_t)i * N;
    uint64_t x = a.x[b * a.x_bstride + off + c];
    uint64_t z = a.z[b * a.z_bstride + off + c];
    uint64_t r = mul_shoup(x + q - z, pi.w, pi.wp, q);
    if (a.add && ((a.add_mask >> b) & 1)) {
        uint32_t sc = (a.add_galois != 1) ? aut_eval_src(c, a.add_galois, a.n) : c;
        r = add_mod(r, a.add[b * a.add_pstride + off + sc], q);
    }
    a.out[b * a.out_bstride + off + c] = r;
}

hipError_t launch_moddown_epi(const Ctx &c, const uint64_t *x, const uint64_t *z, uint64_t *out,
                              uint32_t level, const uint64_t *add, uint32_t add_galois,
                              uint32_t add_mask, uint32_t batch, size_t x_bstride, size_t z_bstride,
                              size_t out_bstride, size_t add_pstride, hipStream_t s) {
    MdEpiArgs a{};
    a.x = x;
    a.z = z;
    a.add = add;
    a.out = out;
    a.mc = c.mc;
    a.pinv = c.pinv;
    a.x_bstride = x_bstride;
    a.z_bstride = z_bstride;
    a.out_bstride = out_bstride;
    a.add_pstride = add_pstride;
    a.n = c.log_n;
    a.add_galois = add_galois;
    a.add_mask = add_mask;
    dim3 grid((c.n + 255) / 256, batch, level);
    ProfScope ps(c, HKS_K_MODDOWN_EPI, s);
    hipLaunchKernelGGL(moddown_epi_kernel, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ elementwise

struct EwArgs {
    const uint64_t *x, *y, *z, *w;
    uint64_t *out;
    const ModC *mc;
    const Shoup *sh;
    const uint64_t *hv;
    uint32_t n, level, n_poly;
    size_t xs, ys, outs;
};

// PtMult (Algorithm 1, line 2): out[p][l] = ct[p][l] * pt[l].
__global__ void __launch_bounds__(256) mulpt_kernel(const EwArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t l = blockIdx.z, p = blockIdx.y;
    if (c >= N) return;
    const ModC m = a.mc[l];
    const size_t o = ((size_t)p * a.level + l) * N + c;
    a.out[o] = mul_mod(a.x[o], a.y[(size_t)l * N + c], m.q, m.mu);
}

// Tensor product (Algorithm 2, line 3): (a1 a2, a1 b2 + a2 b1, b1 b2).
__global__ void __launch_bounds__(256) tensor_kernel(const EwArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t l = blockIdx.z;
    if (c >= N) return;
    const ModC m = a.mc[l];
    const size_t o = (size_t)l * N + c, pl = (size_t)a.level * N;
    uint64_t a1 = a.x[o], b1 = a.x[pl + o], a2 = a.y[o], b2 = a.y[pl + o];
    a.out[o] = mul_mod(a1, a2, m.q, m.mu);
    Acc128 acc;
    acc.mac(a1, b2);
    acc.mac(a2, b1);
    a.out[pl + o] = acc.reduce(m.q, m.mu);
    a.out[2 * pl + o] = mul_mod(b1, b2, m.q, m.mu);
}

// out = x + y over n_poly polys of `level` limbs (limb index = flat % level).
__global__ void __launch_bounds__(256) add_kernel(const EwArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t f = blockIdx.z;
    if (c >= N) return;
    const uint64_t q = a.mc[f % a.level].q;
    const size_t o = (size_t)f * N + c;
    a.out[o] = add_mod(a.x[o], a.y[o], q);
}

// Rescale: r = coefficient-form last limb (canonical mod q_last); w_i =
// (r + h - h) mod q_i computed as (r + h mod q_last) - h, i.e. the rounding
// correction of floor((x + h) / q_last) reduced into each remaining limb.
__global__ void __launch_bounds__(256) rescale_prep_kernel(const EwArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t i = blockIdx.z, p = blockIdx.y;
    if (c >= N) return;
    const uint32_t l = a.level;
    const uint64_t ql = a.mc[l - 1].q;
    const uint64_t h = (ql - 1) >> 1;
    uint64_t r = a.x[p * a.xs + c];
    r = add_mod(r, h, ql);                   // (x_last + h) mod q_last
    const ModC m = a.mc[i];
    uint64_t rm = csub(r, m.q);              // r < q_last < 2 q_i
    uint64_t hm = a.hv[(size_t)l * (a.n_poly) + i];
    a.out[p * a.outs + (size_t)i * N + c] = sub_mod(rm, hm, m.q);
}

__global__ void __launch_bounds__(256) rescale_epi_kernel(const EwArgs a) {
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t i = blockIdx.z, p = blockIdx.y;
    if (c >= N) return;
    const uint64_t q = a.mc[i].q;
    const Shoup s = a.sh[(size_t)a.level * a.n_poly + i];
    uint64_t x = a.x[p * a.xs + (size_t)i * N + c];
    uint64_t w = a.y[p * a.ys + (size_t)i * N + c];
    a.out[p * a.outs + (size_t)i * N + c] = mul_shoup(x + q - w, s.w, s.wp, q);
}

hipError_t launch_mulpt(const Ctx &c, const uint64_t *ct, const uint64_t *pt, uint64_t *out,
                        uint32_t level, uint32_t n_poly, hipStream_t s) {
    EwArgs a{};
    a.x = ct;
    a.y = pt;
    a.out = out;
    a.mc = c.mc;
    a.n = c.log_n;
    a.level = level;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(mulpt_kernel, dim3((c.n + 255) / 256, n_poly, level), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tensor(const Ctx &c, const uint64_t *ct1, const uint64_t *ct2, uint64_t *out3,
                         uint32_t level, hipStream_t s) {
    EwArgs a{};
    a.x = ct1;
    a.y = ct2;
    a.out = out3;
    a.mc = c.mc;
    a.n = c.log_n;
    a.level = level;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(tensor_kernel, dim3((c.n + 255) / 256, 1, level), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_add(const Ctx &c, const uint64_t *x, const uint64_t *y, uint64_t *out,
                      uint32_t n_limbs_total, uint32_t level, hipStream_t s) {
    EwArgs a{};
    a.x = x;
    a.y = y;
    a.out = out;
    a.mc = c.mc;
    a.n = c.log_n;
    a.level = level;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(add_kernel, dim3((c.n + 255) / 256, 1, n_limbs_total), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_rescale_prep(const Ctx &c, const uint64_t *rlast, uint64_t *w, uint32_t level,
                               uint32_t n_poly, size_t r_bstride, size_t w_bstride, hipStream_t s) {
    EwArgs a{};
    a.x = rlast;
    a.out = w;
    a.mc = c.mc;
    a.hv = c.rs_h;
    a.n = c.log_n;
    a.level = level;
    a.n_poly = c.L;  // row stride of the per-level table
    a.xs = r_bstride;
    a.outs = w_bstride;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(rescale_prep_kernel, dim3((c.n + 255) / 256, n_poly, level - 1), dim3(256), 0,
                       s, a);
    return hipGetLastError();
}

hipError_t launch_rescale_epi(const Ctx &c, const uint64_t *x, const uint64_t *w, uint64_t *out,
                              uint32_t level, uint32_t n_poly, size_t x_bstride, size_t w_bstride,
                              size_t out_bstride, hipStream_t s) {
    EwArgs a{};
    a.x = x;
    a.y = w;
    a.out = out;
    a.mc = c.mc;
    a.sh = c.rs_qinv;
    a.n = c.log_n;
    a.level = level;
    a.n_poly = c.L;
    a.xs = x_bstride;
    a.ys = w_bstride;
    a.outs = out_bstride;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(rescale_epi_kernel, dim3((c.n + 255) / 256, n_poly, level - 1), dim3(256), 0,
                       s, a);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) copy_kernel(const uint64_t *in, uint64_t *out, size_t words) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) out[i] = in[i];
}

hipError_t launch_copy(const uint64_t *in, uint64_t *out, size_t words, hipStream_t s) {
    if (!words) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, words);
    return hipGetLastError();
}

}  // namespace hks
