// KSKInnerProd fused with ModUp's last forward pass and ModDown's first
// inverse pass (the key-switch kernel), and PtMatVecMult with one ModDown
// (Sec. 4-5 of the paper recast for LDS; building blocks in ntt_device.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
#include "hks_internal.h"
#include "modarith.h"
#include "ntt_device.h"

namespace hks {

// ------------------------------------------------------------------ KSKInnerProd (+ ModUp's last pass, + ModDown's first)


struct KskRowArgs {
    KskBatch kb;             // per ciphertext: own-digit source, key [dnum][2][L+K][N], galois
    const uint64_t *ext;     // [beta][E][N] converted limbs: after the forward column pass (rowpass) or in evaluation form
    uint64_t *uq;            // [2][level][N] KSKInnerProd on the q limbs
    uint64_t *pc;            // [2][K][N] P limbs after the inverse row pass
    const Shoup *twf, *twi;
    const uint64_t *twmf, *twmi;  // the tables in Montgomery form
    const ModC *mc;
    const Shoup *pmod;  // NewMult: [P]_{q_i}
    size_t dstride, ext_bstride, uq_bstride, pc_bstride;
    uint32_t n, n1, n2, L, K, alpha, all_direct, keyidx, nb, xcd_group, pck;
    uint32_t level0, uniform;  // every entry at level0 (uniform), else kb.level[b]
};

// The forward row twiddles (Montgomery form) of the block's rows, staged in
// LDS by each wave for the wave's own lines (line = threadIdx.x / T; a
// wave's LDS operations take effect in order, so its threads read them
// without a barrier): line l's S entries hold at [0, 2) the aligned pair
// around its stage-0 entry (2^n1 + row) and at [2^ls, 2^(ls+1)) the 2^ls
// entries ((2^n1 + row) << ls) + m of stage ls >= 1; each lane copies E/2 of
// the wave's 16-byte chunks.
template <int LOGS, int E, int NT>
__device__ __forceinline__ void row_twiddle_stage(uint64_t *twbuf, const uint64_t *tw, uint32_t row0, uint32_t n1) {
    constexpr int S = 1 << LOGS, T = S / E, W = NT < 64 ? NT : 64, CPL = S / 2;
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t line0 = wave * 64 / T;  // the wave's first line
    ulonglong2 v[E / 2];
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
        const uint32_t g = i * W + lane;  // chunk within the wave's lines
        const uint32_t l = line0 + g / CPL, cc = g % CPL;
        const uint32_t hi = (1u << n1) + row0 + l;
        size_t src;
        if (cc == 0) {
            src = hi & ~1u;
        } else {
            const uint32_t e = 2 * cc, ls = 31 - __builtin_clz(e);
            src = ((size_t)hi << ls) + (e - (1u << ls));
        }
        v[i] = *reinterpret_cast<const ulonglong2 *>(tw + src);
    }
    ulonglong2 *dst = reinterpret_cast<ulonglong2 *>(twbuf) + (size_t)line0 * CPL;
#pragma unroll
    for (int i = 0; i < E / 2; ++i) dst[i * W + lane] = v[i];
    wave_sync();
}
// Twiddles from row_twiddle_stage's buffer for one line.
struct TwRowsLdsM {
    const uint64_t *tw;  // the line's S entries in LDS
    uint32_t odd;        // row & 1: the stage-0 entry's place in its pair
    __device__ __forceinline__ uint64_t operator()(int ls, uint32_t m) const {
        return ls == 0 ? tw[odd] : tw[(1u << ls) + m];
    }
};

// One block = one target limb t of Q_level U P and ROW_LINES rows, in the
// row-pass layout (each thread E elements of one row; every launch takes
// E = 8).  For each digit j:
// the converted limb x_{j,t} gets the forward row pass on chip (ROWPASS: the
// last pass of ModUp's NTT; lazy values < 2^56), or the digit's own limb is
// read from the input through the automorph; then u_t += x ksk[j][0][t],
// v_t += x ksk[j][1][t] (Barrett products of the lazy value and the key,
// canonical sums).  q limbs store (u_t, v_t); special-prime limbs run
// ModDown's inverse row pass on both in registers before storing (the
// forward pass ends in the layout the inverse pass starts from).
// Register budget: with LZ (lazy 128-bit sums, 8 elements per thread) the
// row-pass form needs two waves per SIMD and the direct form fits three;
// without LZ (a reduction per digit, half the accumulator registers) both
// fit three.  Row-pass launches go without LZ (measured against lazy sums:
// batched KSKInnerProd -5%, a single Rotate -1%, with the twiddles from LDS
// and per-wave row synchronization); the direct form and NewMult keep LZ.
template <int LOGS, bool ROWPASS, int E, bool SEEDED, bool NM, bool LZ = true>
__global__ void __launch_bounds__((Tile<LOGS, ROW_LINES, false, E>::NT))
__attribute__((amdgpu_waves_per_eu(E == 8 ? ((LZ && ROWPASS) ? 2 : 3) : 2)))
ksk_rows_kernel(const KskRowArgs a) {
    using TL = Tile<LOGS, ROW_LINES, false, E>;
    using IOF = IoLayout<LOGS, true, E>;
    using IOI = IoLayout<LOGS, false, E>;
    static_assert(IOF::OUT_LO == IOI::IN_LO && IOF::OUT_HI == IOI::IN_HI, "row-pass layouts must chain");
    __shared__ uint64_t lds[TL::WORDS];
    // direct digits (hoisted rotations): the special limbs' inverse row-pass
    // twiddles for the block's ROW_LINES rows (every stage), staged once for
    // u's and v's passes (measured: HRotate +2%)
    __shared__ Shoup lds_tw[(ROWPASS || LOGS > 8) ? 1 : ROW_LINES * ((1 << LOGS) - 1)];
    // the row-pass form with passes of 8 or more stages: Montgomery-form
    // twiddles (half the bytes of a Shoup pair), the forward ones staged in
    // LDS once (the same for every digit).  Measured against Shoup pairs
    // from the global table: Rotate -2%, ksk -5%; batched launches -7% per
    // launch.  Shorter passes read Shoup pairs from the table.
    constexpr bool MT = ROWPASS && MONT_ROWS<LOGS>;
    __shared__ __attribute__((aligned(16))) uint64_t twbuf[MT ? ROW_LINES * (1 << LOGS) : 2];
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
    constexpr bool LAZY = E == 8 && LZ;
    uint64_t u[E], v[E];
    Acc128 ua[LAZY ? E : 1], va[LAZY ? E : 1];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = v[e] = 0;
    bool lds_used = false;
    if constexpr (MT) row_twiddle_stage<LOGS, E, TL::NT>(twbuf, a.twmf + (size_t)mod * N, tile * ROW_LINES, a.n1);
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
                if (lds_used) pass_sync<false>();
                if constexpr (MT) {
                    pass_regs<LOGS, ROW_LINES, false, true, false, E>(
                        true, xv, lds, line, t, q, mcv.nq, TwRowsLdsM{twbuf + (size_t)line * (1 << LOGS), lg & 1u},
                        LastInv{}, mcv.qi);
                } else {
                    pass_regs<LOGS, ROW_LINES, false, true, false, E>(true, xv, lds, line, t, q, mcv.nq,
                                                                      TwRows{a.twf + (size_t)mod * N, lg, a.n1},
                                                                      LastInv{});
                }
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
    if (lds_used) pass_sync<false>();
    if constexpr (MT) {
        const TwRowsM twi{a.twmi + (size_t)mod * N, lg, a.n1};
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, u, lds, line, t, q, mcv.nq, twi, LastInv{},
                                                           mcv.qi);
        gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(u, pc + (size_t)kp * N, t, lg, a.n2);
        pass_sync<false>();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, v, lds, line, t, q, mcv.nq, twi, LastInv{},
                                                           mcv.qi);
    } else if constexpr (ROWPASS || LOGS > 8) {
        const TwRows twi{a.twi + (size_t)mod * N, lg, a.n1};
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, u, lds, line, t, q, mcv.nq, twi, LastInv{});
        gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(u, pc + (size_t)kp * N, t, lg, a.n2);
        pass_sync<false>();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, v, lds, line, t, q, mcv.nq, twi, LastInv{});
    } else {
        const TwRowsLds<ROW_LINES> twl{lds_tw, (uint32_t)line};
        stage_row_twiddles<LOGS, ROW_LINES>(lds_tw, a.twi + (size_t)mod * N, tile * ROW_LINES, a.n1);
        __syncthreads();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, u, lds, line, t, q, mcv.nq, twl, LastInv{});
        gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(u, pc + (size_t)kp * N, t, lg, a.n2);
        pass_sync<false>();
        pass_regs<LOGS, ROW_LINES, false, false, false, E>(true, v, lds, line, t, q, mcv.nq, twl, LastInv{});
    }
    gstore<LOGS, false, IOI::OUT_LO, IOI::OUT_HI, E>(v, pc + ((size_t)a.pck + kp) * N, t, lg, a.n2);
}

template <bool ROWPASS, int E, bool SEEDED, bool NM = false, bool LZ = true>
static hipError_t launch_ksk_rows_t(const KskRowArgs &a, uint32_t n2, dim3 grid, hipStream_t s) {
    switch (n2) {
        case 5: hipLaunchKernelGGL((ksk_rows_kernel<5, ROWPASS, E, SEEDED, NM, LZ>), grid, dim3(Tile<5, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 6: hipLaunchKernelGGL((ksk_rows_kernel<6, ROWPASS, E, SEEDED, NM, LZ>), grid, dim3(Tile<6, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 7: hipLaunchKernelGGL((ksk_rows_kernel<7, ROWPASS, E, SEEDED, NM, LZ>), grid, dim3(Tile<7, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 8: hipLaunchKernelGGL((ksk_rows_kernel<8, ROWPASS, E, SEEDED, NM, LZ>), grid, dim3(Tile<8, ROW_LINES, false, E>::NT), 0, s, a); break;
        case 9: hipLaunchKernelGGL((ksk_rows_kernel<9, ROWPASS, E, SEEDED, NM, LZ>), grid, dim3(Tile<9, ROW_LINES, false, E>::NT), 0, s, a); break;
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
    a.twmf = c.twm_fwd;
    a.twmi = c.twm_inv;
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
    // a seeded key's rows a_j are generated in the kernel; launches with the
    // row pass reduce per digit (three waves per SIMD)
    if (kb.seeded) {
        if (!rowpass) return launch_ksk_rows_t<false, 8, true>(a, c.n2, grid, s);
        return launch_ksk_rows_t<true, 8, true, false, false>(a, c.n2, grid, s);
    }
    if (!rowpass) return launch_ksk_rows_t<false, 8, false>(a, c.n2, grid, s);
    return launch_ksk_rows_t<true, 8, false, false, false>(a, c.n2, grid, s);
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
    pass_sync<false>();
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
        case 9: hipLaunchKernelGGL((ksk_matvec_kernel<9, 8>), grid, dim3(Tile<9, ROW_LINES, false, 8>::NT), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hks
