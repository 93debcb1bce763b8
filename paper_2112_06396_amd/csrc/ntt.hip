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
//   IO_CONV   column pass whose load computes NewLimb (the basis conversion
//             of ModUp / ModDown) from the digit's coefficient-form limbs, so
//             the converted limb is produced on chip and goes straight into
//             its NTT (alpha-limb caching);
//   rows_ksk  row pass of every digit of one target limb followed by
//             KSKInnerProd against the key, so extended digits never reach
//             HBM in evaluation form; for the special-prime limbs it then
//             runs the inverse row pass of ModDown (P limbs first);
//   IO_MDEPI  row pass of the ModDown correction followed by
//             (u - z) * P^-1 (+ the automorphed b of Rotate).
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "hks_internal.h"
#include "modarith.h"

namespace hks {

template <int LOGS, int LINES, bool COLS>
struct Tile {
    static constexpr int S = 1 << LOGS;
    static constexpr int T = S / 16;         // threads per line
    static constexpr int NT = LINES * T;     // threads per block
    static constexpr int EPT = 16;           // elements per thread
    static constexpr int ROWP = S + S / 16;  // padded row length (row tiles)
    static constexpr int COLP = LINES + 1;   // padded k-row length (column tiles)
    static constexpr int WORDS = COLS ? S * COLP : LINES * ROWP;
    __device__ static __forceinline__ int idx(int line, int k) {
        return COLS ? k * COLP + line : line * ROWP + k + (k >> 4);
    }
};

// One phase over bits [LO, HI) of the sub-index k.  Twiddle of the butterfly
// on bit `bit` for lower element k:
//   column pass: index 2^s + (k >> (bit+1)),           s = LOGS-1-bit;
//   row pass:    index 2^s + (r << (LOGS-1-bit)) + (k >> (bit+1)),
//                s = n1 + LOGS-1-bit, r the row.
// Elements whose k agree above `bit` share the twiddle, so each stage loads
// 16 >> (vb+1) twiddles per thread.
template <int LOGS, int LINES, bool COLS, bool FWD, int LO, int HI>
__device__ __forceinline__ void ntt_phase(uint64_t *lds, int line, int t, uint32_t row, uint32_t n1, uint64_t q,
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
        const int ls = LOGS - 1 - bit;  // stage within this pass
        const bool fold_stage = !FWD && COLS && ls == 0;
        const uint32_t sbase = COLS ? (1u << ls) : ((1u << n1) << ls);
        Shoup wc[8];
#pragma unroll
        for (int key = 0; key < 8; ++key) {
            if (key < (16 >> (vb + 1)) && !fold_stage) {
                const uint32_t k = (uint32_t)kk[key << (vb + 1)];
                const uint32_t ix = COLS ? (sbase + (k >> (bit + 1)))
                                         : (sbase + (row << ls) + (k >> (bit + 1)));
                wc[key] = tw[ix];
            }
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            if ((e >> vb) & 1) continue;
            const int e2 = e + (1 << vb);
            const Shoup w = wc[(e >> (vb + 1)) & 7];
            if (FWD) {
                const uint64_t u = x[e];
                const uint64_t tv = mul_shoup_lazy(x[e2], w.w, w.wp, q);
                x[e] = u + tv;
                x[e2] = u + q2 - tv;
            } else {
                const uint64_t u = x[e], v = x[e2];
                if (fold_stage) {
                    x[e] = mul_shoup(u + v, fold.c.w, fold.c.wp, q);
                    x[e2] = mul_shoup(u + q2 - v, fold.cw.w, fold.cw.wp, q);
                } else {
                    x[e] = csub(u + v, q2);
                    x[e2] = mul_shoup_lazy(u + q2 - v, w.w, w.wp, q);
                }
            }
        }
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) lds[TL::idx(line, kk[e])] = x[e];
}

// All phases of one pass on the LDS tile (caller synchronizes before/after).
template <int LOGS, int LINES, bool COLS, bool FWD>
__device__ __forceinline__ void ntt_tile(uint64_t *lds, int line, int t, uint32_t row, uint32_t n1, uint64_t q,
                                         const Shoup *__restrict__ tw, const LastInv &fold) {
    constexpr int P0L = LOGS - 4;
    constexpr int P1H = P0L, P1L = (P0L - 4) > 0 ? (P0L - 4) : 0;
    constexpr int P2H = P1L, P2L = 0;
    static_assert(LOGS >= 5 && LOGS <= 12, "sub-transform size");
    if (FWD) {
        ntt_phase<LOGS, LINES, COLS, true, P0L, LOGS>(lds, line, t, row, n1, q, tw, fold);
        __syncthreads();
        ntt_phase<LOGS, LINES, COLS, true, P1L, P1H>(lds, line, t, row, n1, q, tw, fold);
        if constexpr (P2H > P2L) {
            __syncthreads();
            ntt_phase<LOGS, LINES, COLS, true, P2L, P2H>(lds, line, t, row, n1, q, tw, fold);
        }
    } else {
        if constexpr (P2H > P2L) {
            ntt_phase<LOGS, LINES, COLS, false, P2L, P2H>(lds, line, t, row, n1, q, tw, fold);
            __syncthreads();
        }
        ntt_phase<LOGS, LINES, COLS, false, P1L, P1H>(lds, line, t, row, n1, q, tw, fold);
        __syncthreads();
        ntt_phase<LOGS, LINES, COLS, false, P0L, LOGS>(lds, line, t, row, n1, q, tw, fold);
    }
}

// All phases of one pass with the work of each phase done only where
// `active` holds; every thread of the block reaches every barrier, so thread
// groups of one block may run passes on different tiles (or sit one out).
template <int LOGS, int LINES, bool COLS, bool FWD>
__device__ __forceinline__ void ntt_tile_guarded(bool active, uint64_t *lds, int line, int t, uint32_t row,
                                                 uint32_t n1, uint64_t q, const Shoup *__restrict__ tw,
                                                 const LastInv &fold) {
    constexpr int P0L = LOGS - 4;
    constexpr int P1H = P0L, P1L = (P0L - 4) > 0 ? (P0L - 4) : 0;
    constexpr int P2H = P1L, P2L = 0;
    if (FWD) {
        if (active) ntt_phase<LOGS, LINES, COLS, true, P0L, LOGS>(lds, line, t, row, n1, q, tw, fold);
        __syncthreads();
        if (active) ntt_phase<LOGS, LINES, COLS, true, P1L, P1H>(lds, line, t, row, n1, q, tw, fold);
        if constexpr (P2H > P2L) {
            __syncthreads();
            if (active) ntt_phase<LOGS, LINES, COLS, true, P2L, P2H>(lds, line, t, row, n1, q, tw, fold);
        }
    } else {
        if constexpr (P2H > P2L) {
            if (active) ntt_phase<LOGS, LINES, COLS, false, P2L, P2H>(lds, line, t, row, n1, q, tw, fold);
            __syncthreads();
        }
        if (active) ntt_phase<LOGS, LINES, COLS, false, P1L, P1H>(lds, line, t, row, n1, q, tw, fold);
        __syncthreads();
        if (active) ntt_phase<LOGS, LINES, COLS, false, P0L, LOGS>(lds, line, t, row, n1, q, tw, fold);
    }
}

// thread -> (line, t): column tiles put lines fastest (LDS rows contiguous),
// row tiles put the threads of one line together.
template <int LOGS, int LINES, bool COLS>
__device__ __forceinline__ void thread_coords(int tid, int &line, int &t) {
    using TL = Tile<LOGS, LINES, COLS>;
    if (COLS) {
        line = tid % LINES;
        t = tid / LINES;
    } else {
        t = tid % TL::T;
        line = tid / TL::T;
    }
}

// element e of the tile (cooperative, coalesced pattern) -> (line, k, j)
template <int LOGS, int LINES, bool COLS>
__device__ __forceinline__ void elem_coords(int e, uint32_t line0, uint32_t n2, int &line, int &k, uint32_t &j) {
    using TL = Tile<LOGS, LINES, COLS>;
    if (COLS) {
        k = e / LINES;
        line = e % LINES;
        j = ((uint32_t)k << n2) + line0 + line;
    } else {
        line = e / TL::S;
        k = e % TL::S;
        j = ((line0 + line) << n2) + k;
    }
}

struct NttArgs {
    const Ctx *ctx;  // host-side only (timing); not read by kernels
    const uint64_t *in;
    uint64_t *out;
    const Shoup *tw;      // [M][N] forward or inverse table
    const ModC *mc;
    const LastInv *li;    // folded last inverse stage, indexed by cidx
    const uint64_t *conv; // IO_CONV: constant rows, row cidx at conv + cidx * cstride
    const uint64_t *uq;   // IO_MDEPI: u limbs (limb cidx), batch stride uq_bstride
    const Shoup *pinv;    // IO_MDEPI: P^-1 mod q_i
    const uint64_t *add;  // IO_MDEPI: addend (limb cidx) for polys selected by add_mask
    size_t in_bstride, out_bstride, uq_bstride, add_pstride;
    uint32_t n, n1, n2, galois, cstride, add_galois, add_mask;
    LimbMap m;
};

enum { IO_PLAIN = 0, IO_GATHER = 1, IO_REDUCE = 2, IO_CONV = 3, IO_MDEPI = 4 };

template <int LOGS, int LINES, bool COLS, bool FWD, int IO>
__global__ void __launch_bounds__((Tile<LOGS, LINES, COLS>::NT)) ntt_pass_kernel(const NttArgs a) {
    using TL = Tile<LOGS, LINES, COLS>;
    __shared__ uint64_t lds[TL::WORDS];
    const uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
    const uint32_t tiles = lines_per_limb / LINES;
    const uint32_t li = blockIdx.x / tiles;
    const uint32_t tile = blockIdx.x % tiles;
    const uint32_t b = blockIdx.y;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = a.m.mod[li];
    const ModC mcv = a.mc[mod];
    const uint64_t q = mcv.q;
    const uint64_t *src = a.in + b * a.in_bstride + (size_t)a.m.in_off[li] * N;
    uint64_t *dst = a.out + b * a.out_bstride + (size_t)a.m.out_off[li] * N;
    const Shoup *tw = a.tw + (size_t)mod * N;
    const int tid = threadIdx.x;
    const uint32_t line0 = tile * LINES;

    if (IO == IO_CONV) {
        // NewLimb: out = sum_i y_i * K_i mod q over the digit's n_src limbs,
        // CH elements at a time so that their source loads overlap
        constexpr int MAXS = 16, CH = 4;
        const uint32_t ns = a.m.nsrc[li];
        const uint64_t *kr = a.conv + (size_t)a.m.cidx[li] * a.cstride;
        uint64_t kc[MAXS];
#pragma unroll
        for (int i = 0; i < MAXS; ++i) kc[i] = (i < (int)ns) ? kr[i] : 0;
#pragma unroll 1
        for (int i0 = 0; i0 < TL::EPT; i0 += CH) {
            uint32_t jj[CH];
            int ii[CH];
            MacAcc acc[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                int line, k;
                elem_coords<LOGS, LINES, COLS>(tid + (i0 + c) * TL::NT, line0, a.n2, line, k, jj[c]);
                ii[c] = TL::idx(line, k);
            }
#pragma unroll
            for (int i = 0; i < MAXS; ++i) {
                if (i < (int)ns) {
                    uint64_t yv[CH];
#pragma unroll
                    for (int c = 0; c < CH; ++c) yv[c] = src[(size_t)i * N + jj[c]];
#pragma unroll
                    for (int c = 0; c < CH; ++c) acc[c].mac(yv[c], kc[i]);
                }
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) lds[ii[c]] = acc[c].reduce(q, mcv.mu);
        }
    } else {
        uint64_t v[TL::EPT];
#pragma unroll
        for (int i = 0; i < TL::EPT; ++i) {
            int line, k;
            uint32_t j;
            elem_coords<LOGS, LINES, COLS>(tid + i * TL::NT, line0, a.n2, line, k, j);
            const uint32_t sj = (IO == IO_GATHER) ? aut_eval_src(j, a.galois, a.n) : j;
            v[i] = src[sj];
        }
#pragma unroll
        for (int i = 0; i < TL::EPT; ++i) {
            int line, k;
            uint32_t j;
            elem_coords<LOGS, LINES, COLS>(tid + i * TL::NT, line0, a.n2, line, k, j);
            lds[TL::idx(line, k)] = v[i];
        }
    }
    __syncthreads();

    int line, t;
    thread_coords<LOGS, LINES, COLS>(tid, line, t);
    const LastInv fold = (!FWD && COLS) ? a.li[a.m.cidx[li]] : LastInv{};
    ntt_tile<LOGS, LINES, COLS, FWD>(lds, line, t, line0 + line, a.n1, q, tw, fold);
    __syncthreads();

    if (IO == IO_MDEPI) {
        const uint32_t ui = a.m.cidx[li];
        const uint64_t *u = a.uq + b * a.uq_bstride + (size_t)ui * N;
        const Shoup pi = a.pinv[ui];
        const bool do_add = a.add && ((a.add_mask >> b) & 1u);
        const uint64_t *ad = do_add ? a.add + b * a.add_pstride + (size_t)ui * N : nullptr;
#pragma unroll 4
        for (int i = 0; i < TL::EPT; ++i) {
            int ln, k;
            uint32_t j;
            elem_coords<LOGS, LINES, COLS>(tid + i * TL::NT, line0, a.n2, ln, k, j);
            const uint64_t z = reduce64(lds[TL::idx(ln, k)], q, mcv.mu);
            uint64_t r = mul_shoup(u[j] + q - z, pi.w, pi.wp, q);
            if (do_add) r = add_mod(r, ad[a.add_galois != 1 ? aut_eval_src(j, a.add_galois, a.n) : j], q);
            dst[j] = r;
        }
    } else {
#pragma unroll
        for (int i = 0; i < TL::EPT; ++i) {
            int ln, k;
            uint32_t j;
            elem_coords<LOGS, LINES, COLS>(tid + i * TL::NT, line0, a.n2, ln, k, j);
            uint64_t v = lds[TL::idx(ln, k)];
            if (IO == IO_REDUCE) v = reduce64(v, q, mcv.mu);
            dst[j] = v;
        }
    }
}

constexpr int COL_LINES = 16;
constexpr int ROW_LINES = 8;

template <int LOGS, bool COLS, bool FWD, int IO>
static hipError_t launch_pass_t(const NttArgs &a, uint32_t count, uint32_t batch, hipStream_t s) {
    constexpr int LINES = COLS ? COL_LINES : ROW_LINES;
    using TL = Tile<LOGS, LINES, COLS>;
    ProfScope ps(*a.ctx, FWD ? (COLS ? HKS_K_NTT_FWD_COLS : HKS_K_NTT_FWD_ROWS)
                             : (COLS ? HKS_K_NTT_INV_COLS : HKS_K_NTT_INV_ROWS), s);
    const uint32_t lines_per_limb = 1u << (COLS ? a.n2 : a.n1);
    dim3 grid(count * (lines_per_limb / LINES), batch);
    hipLaunchKernelGGL((ntt_pass_kernel<LOGS, LINES, COLS, FWD, IO>), grid, dim3(TL::NT), 0, s, a);
    return hipGetLastError();
}

template <bool COLS, bool FWD, int IO>
static hipError_t dispatch_pass(const NttArgs &a, int logs, uint32_t count, uint32_t batch, hipStream_t s) {
    switch (logs) {
        case 5: return launch_pass_t<5, COLS, FWD, IO>(a, count, batch, s);
        case 6: return launch_pass_t<6, COLS, FWD, IO>(a, count, batch, s);
        case 7: return launch_pass_t<7, COLS, FWD, IO>(a, count, batch, s);
        case 8: return launch_pass_t<8, COLS, FWD, IO>(a, count, batch, s);
        default: return hipErrorInvalidValue;
    }
}

static NttArgs base_args(const Ctx &c, const LimbMap &m, bool fwd) {
    NttArgs a{};
    a.ctx = &c;
    a.tw = fwd ? c.tw_fwd : c.tw_inv;
    a.mc = c.mc;
    a.li = c.li_plain;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.galois = 1;
    a.m = m;
    return a;
}

static void outputs_as_inputs(NttArgs &a, const LimbMap &m) {
    for (uint32_t i = 0; i < m.count; ++i) a.m.in_off[i] = m.out_off[i];
}

hipError_t launch_ntt_fwd(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out, uint32_t batch,
                          size_t in_bstride, size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, true);
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    hipError_t e = dispatch_pass<true, true, IO_PLAIN>(a, c.n1, m.count, batch, s);
    if (e != hipSuccess) return e;
    a.in = out;
    a.in_bstride = out_bstride;
    outputs_as_inputs(a, m);
    return dispatch_pass<false, true, IO_REDUCE>(a, c.n2, m.count, batch, s);
}

hipError_t launch_ntt_fwd_rows(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                               uint32_t batch, size_t in_bstride, size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, true);
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    return dispatch_pass<false, true, IO_REDUCE>(a, c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out, const LastInv *li,
                          uint32_t galois, uint32_t batch, size_t in_bstride, size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, false);
    a.li = li;
    a.galois = galois;
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    hipError_t e = (galois != 1) ? dispatch_pass<false, false, IO_GATHER>(a, c.n2, m.count, batch, s)
                                 : dispatch_pass<false, false, IO_PLAIN>(a, c.n2, m.count, batch, s);
    if (e != hipSuccess) return e;
    a.in = out;
    a.in_bstride = out_bstride;
    a.galois = 1;
    outputs_as_inputs(a, m);
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

hipError_t launch_ntt_inv_rows(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                               uint32_t batch, size_t in_bstride, size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, false);
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    return dispatch_pass<false, false, IO_PLAIN>(a, c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv_cols(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                               const LastInv *li, uint32_t batch, size_t in_bstride, size_t out_bstride,
                               hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, false);
    a.li = li;
    a.in = in;
    a.out = out;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

hipError_t launch_conv_cols(const Ctx &c, const LimbMap &m, const uint64_t *y, const uint64_t *conv,
                            uint32_t cstride, uint64_t *out, uint32_t batch, size_t in_bstride,
                            size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, true);
    a.in = y;
    a.out = out;
    a.conv = conv;
    a.cstride = cstride;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    return dispatch_pass<true, true, IO_CONV>(a, c.n1, m.count, batch, s);
}

hipError_t launch_rows_mdepi(const Ctx &c, const LimbMap &m, const uint64_t *zc, uint64_t *out,
                             const uint64_t *uq, size_t uq_bstride, const uint64_t *add, uint32_t add_galois,
                             uint32_t add_mask, size_t add_pstride, uint32_t batch, size_t in_bstride,
                             size_t out_bstride, hipStream_t s) {
    if (m.count == 0 || batch == 0) return hipSuccess;
    NttArgs a = base_args(c, m, true);
    a.in = zc;
    a.out = out;
    a.uq = uq;
    a.uq_bstride = uq_bstride;
    a.pinv = c.pinv;
    a.add = add;
    a.add_galois = add_galois;
    a.add_mask = add_mask;
    a.add_pstride = add_pstride;
    a.in_bstride = in_bstride;
    a.out_bstride = out_bstride;
    return dispatch_pass<false, true, IO_MDEPI>(a, c.n2, m.count, batch, s);
}

// ------------------------------------------------------------------ row pass + KSKInnerProd

struct KskRowArgs {
    const uint64_t *colout;  // [beta][E][N] column-pass outputs of the new limbs
    const uint64_t *direct;  // evaluation-form digits: limb t of digit j at direct + j*dstride + t*N
    const uint64_t *ksk;     // [dnum][2][L+K][N]
    uint64_t *uq;            // [2][level][N] KSKInnerProd on the q limbs
    uint64_t *pc;            // [2][K][N] P limbs after the inverse row pass
    const Shoup *twf, *twi;
    const ModC *mc;
    size_t dstride;
    uint32_t n, n1, n2, level, L, K, E, alpha, beta, galois, all_direct;
};

// One block = one target limb t of Q_level U P and ROW_LINES rows, DG thread
// groups.  A round handles digits j0..j0+DG-1: group g runs the row pass of
// the converted limb of digit j0+g in its LDS tile (the digit's own limb is
// instead read in evaluation form, gathered through the automorph).  Then
// every thread accumulates, per element, u_t = sum_j x_j ksk[j][0] and
// v_t = sum_j x_j ksk[j][1] (products reduced by Barrett into canonical
// sums; partial sums of earlier rounds come from the output buffers when
// beta > DG).  q limbs store (u_t, v_t).  Special-prime limbs put (u, v) back
// into LDS tiles 0 and 1 at the element's own slot (only the thread that read
// the slot writes it) and run ModDown's inverse row pass on both.
template <int LOGS, int DG>
__global__ void __launch_bounds__((DG * Tile<LOGS, ROW_LINES, false>::NT)) rows_ksk_kernel(const KskRowArgs a) {
    using TL = Tile<LOGS, ROW_LINES, false>;
    constexpr int TW = ROW_LINES * TL::S;  // elements of the tile
    constexpr int BT = DG * TL::NT;        // threads of the block
    constexpr int NTILE = DG < 2 ? 2 : DG;
    __shared__ uint64_t lds[NTILE][TL::WORDS];
    const uint32_t tiles = (1u << a.n1) / ROW_LINES;
    const uint32_t tgt = blockIdx.x / tiles;
    const uint32_t tile = blockIdx.x % tiles;
    const uint32_t N = 1u << a.n;
    const uint32_t mod = tgt < a.level ? tgt : a.L + (tgt - a.level);
    const ModC mcv = a.mc[mod];
    const uint64_t q = mcv.q;
    const int tid = threadIdx.x;
    const int grp = tid / TL::NT, ltid = tid % TL::NT;
    const uint32_t line0 = tile * ROW_LINES;
    const size_t KL = (size_t)a.L + a.K;
    const uint32_t own = (tgt < a.level) ? tgt / a.alpha : 0xffffffffu;
    const bool is_p = tgt >= a.level;
    const uint32_t kp = tgt - a.level;
    uint64_t *ou = is_p ? a.pc + (size_t)kp * N : a.uq + (size_t)tgt * N;
    uint64_t *ov = is_p ? a.pc + ((size_t)a.K + kp) * N : a.uq + ((size_t)a.level + tgt) * N;
    const Shoup *twf = a.twf + (size_t)mod * N;
    int line, t;
    thread_coords<LOGS, ROW_LINES, false>(ltid, line, t);

    for (uint32_t j0 = 0; j0 < a.beta; j0 += DG) {
        const bool last_round = j0 + DG >= a.beta;
        const uint32_t jg = j0 + grp;
        const bool ntt_g = jg < a.beta && !a.all_direct && jg != own;
        if (ntt_g) {
            const uint64_t *src = a.colout + ((size_t)jg * a.E + tgt) * N;
            uint64_t v[TL::EPT];
#pragma unroll
            for (int i = 0; i < TL::EPT; ++i) {
                int ln, k;
                uint32_t j;
                elem_coords<LOGS, ROW_LINES, false>(ltid + i * TL::NT, line0, a.n2, ln, k, j);
                v[i] = src[j];
            }
#pragma unroll
            for (int i = 0; i < TL::EPT; ++i) {
                int ln, k;
                uint32_t j;
                elem_coords<LOGS, ROW_LINES, false>(ltid + i * TL::NT, line0, a.n2, ln, k, j);
                lds[grp][TL::idx(ln, k)] = v[i];
            }
        }
        __syncthreads();
        ntt_tile_guarded<LOGS, ROW_LINES, false, true>(ntt_g, lds[grp], line, t, line0 + line, a.n1, q, twf,
                                                       LastInv{});
        __syncthreads();
        // KSKInnerProd of this round's digits
#pragma unroll 2
        for (int e = tid; e < TW; e += BT) {
            int ln, k;
            uint32_t j;
            elem_coords<LOGS, ROW_LINES, false>(e, line0, a.n2, ln, k, j);
            const int li = TL::idx(ln, k);
            uint64_t u = 0, v = 0;
            if (j0) {
                u = ou[j];
                v = ov[j];
            }
#pragma unroll
            for (int g = 0; g < DG; ++g) {
                const uint32_t jd = j0 + g;
                if (jd >= a.beta) break;
                const uint64_t *k0 = a.ksk + ((size_t)(2 * jd) * KL + mod) * N;
                const uint64_t *k1 = k0 + KL * N;
                uint64_t x;
                if (a.all_direct || jd == own) {
                    const uint64_t *dsrc = a.direct + jd * a.dstride + (size_t)tgt * N;
                    x = dsrc[a.galois != 1 ? aut_eval_src(j, a.galois, a.n) : j];
                } else {
                    x = lds[g][li];
                }
                u = add_mod(u, mul_mod(x, k0[j], q, mcv.mu), q);
                v = add_mod(v, mul_mod(x, k1[j], q, mcv.mu), q);
            }
            if (is_p && last_round) {
                lds[0][li] = u;
                lds[1][li] = v;
            } else {
                ou[j] = u;
                ov[j] = v;
            }
        }
        __syncthreads();
    }
    if (!is_p) return;

    // special-prime limb: inverse row pass (first pass of ModDown's iNTT) of u and v
    const Shoup *twi = a.twi + (size_t)mod * N;
    if (DG >= 2) {
        ntt_tile_guarded<LOGS, ROW_LINES, false, false>(grp < 2, lds[grp < 2 ? grp : 0], line, t, line0 + line,
                                                        a.n1, q, twi, LastInv{});
    } else {
        ntt_tile_guarded<LOGS, ROW_LINES, false, false>(true, lds[0], line, t, line0 + line, a.n1, q, twi,
                                                        LastInv{});
        __syncthreads();
        ntt_tile_guarded<LOGS, ROW_LINES, false, false>(true, lds[1], line, t, line0 + line, a.n1, q, twi,
                                                        LastInv{});
    }
    __syncthreads();
    for (int e = tid; e < TW; e += BT) {
        int ln, k;
        uint32_t j;
        elem_coords<LOGS, ROW_LINES, false>(e, line0, a.n2, ln, k, j);
        const int li = TL::idx(ln, k);
        ou[j] = lds[0][li];
        ov[j] = lds[1][li];
    }
}

hipError_t launch_rows_ksk(const Ctx &c, const uint64_t *colout, const uint64_t *direct, size_t dstride,
                           uint32_t all_direct, const uint64_t *ksk, uint32_t level, uint32_t galois,
                           uint64_t *uq, uint64_t *pc, hipStream_t s) {
    KskRowArgs a{};
    a.colout = colout;
    a.direct = direct;
    a.dstride = dstride;
    a.all_direct = all_direct;
    a.ksk = ksk;
    a.uq = uq;
    a.pc = pc;
    a.twf = c.tw_fwd;
    a.twi = c.tw_inv;
    a.mc = c.mc;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.level = level;
    a.L = c.L;
    a.K = c.K;
    a.E = level + c.K;
    a.alpha = c.alpha;
    a.beta = (level + c.alpha - 1) / c.alpha;
    a.galois = galois;
    ProfScope ps(c, HKS_K_KSK, s);
    const uint32_t tiles = (1u << c.n1) / ROW_LINES;
    dim3 grid(tiles * a.E);
    const uint32_t dg = a.beta >= 4 ? 4 : a.beta;
#define HKS_RK(LG, D) hipLaunchKernelGGL((rows_ksk_kernel<LG, D>), grid, dim3(D * Tile<LG, ROW_LINES, false>::NT), 0, s, a)
#define HKS_RK_DG(LG)       \
    switch (dg) {           \
        case 1: HKS_RK(LG, 1); break; \
        case 2: HKS_RK(LG, 2); break; \
        case 3: HKS_RK(LG, 3); break; \
        default: HKS_RK(LG, 4); break; \
    }
    switch (c.n2) {
        case 5: HKS_RK_DG(5); break;
        case 6: HKS_RK_DG(6); break;
        case 7: HKS_RK_DG(7); break;
        case 8: HKS_RK_DG(8); break;
        default: return hipErrorInvalidValue;
    }
#undef HKS_RK_DG
#undef HKS_RK
    return hipGetLastError();
}

}  // namespace hks
