// HIP kernels for gfx950 besides the NTT passes: standalone KSKInnerProd and
// ModDown final step (used by the single-subroutine ABI calls), Automorph, and
// the elementwise steps of PtMult / Mult (Algorithms 1-2) and Rescale; plus
// the kernel-timing hooks.  The NTT passes and the fused key-switching
// kernels live in ntt.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_util.h"
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
    // timing only (read after the work has finished): no system-scope fence
    // at the record, whose cache writeback and invalidation would land in
    // the measured interval and slow the launch that follows
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
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

// ------------------------------------------------------------------ NewLimb (basis conversion)

struct ConvArgs {
    const uint64_t *in;    // coefficient-form source limbs
    uint64_t *out;
    const uint64_t *conv;  // split constants
    const ModC *mc;
    size_t in_bstride, out_bstride;
    uint32_t n, L, K, alpha, tgroups, keyidx;
    uint32_t level0, coff0;  // every entry's level and constants offset (uniform launches)
    uint32_t coff[MAXB];     // mixed: entry b's constants at conv + coff[b] (its level's table)
    uint8_t lvl[MAXB];       // mixed: entry b's level (MODUP) or number of q targets (ModDown)
};

// Fast basis conversion (NewLimb, Algorithm "ModUp"; also ModDown's step).
// One thread = one coefficient of one digit: its n_src source residues are
// loaded once (split into 25-bit halves) and every target limb of the digit
// is produced from them (the alpha limbs stay on chip for all new limbs).
//   MODUP:   entry b at level lvl[b]; digit j = blockIdx.y / tgroups, sources
//            y[j*alpha .. +n_src), targets t of Q_level U P outside the
//            digit, written at j*E + t (packed, E = level + K) or at
//            j*(L + K) + kappa(t) (keyidx), constants row j*E+t of the
//            entry's level;
//   ModDown: sources the K P limbs, targets the lvl[b] q limbs, out[t],
//            constants row t.
// blockIdx.y % tgroups picks a group of consecutive targets (more blocks for
// a small launch; the groups re-read the sources from L2).  The grid covers
// the launch's largest entry; blocks past an entry's digits leave.
template <bool MODUP, int MAXS, bool MIXED>
__global__ void __launch_bounds__(256) conv_kernel(const ConvArgs a) {
    constexpr int MAXT = 80;  // targets of one digit: level + K <= 64
    __shared__ uint64_t kc[MAXT * MAXS];
    __shared__ ModC mt[MAXT];
    const uint32_t N = 1u << a.n;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t j = blockIdx.y / a.tgroups, grp = blockIdx.y % a.tgroups, b = blockIdx.z;
    const uint32_t level = MIXED ? a.lvl[b] : a.level0;
    const uint32_t lo = MODUP ? j * a.alpha : 0;
    if (MODUP && lo >= level) return;  // the entry has fewer digits
    const uint32_t ns = MODUP ? min(a.alpha, level - lo) : a.K;
    const uint32_t E = level + a.K;
    const uint32_t nt = MODUP ? E : level;
    const uint32_t cstride = MODUP ? a.alpha : a.K;
    const uint32_t ds = a.keyidx ? a.L + a.K : E, pbase = a.keyidx ? a.L : level;
    // the digit's constant rows and target moduli, staged once per block
    const uint64_t *rows = a.conv + (MODUP ? (MIXED ? a.coff[b] : a.coff0) : 0) + (size_t)(MODUP ? j * E : 0) * cstride;
    for (uint32_t i = threadIdx.x; i < nt * MAXS; i += blockDim.x) {
        const uint32_t t = i / MAXS, s = i % MAXS;
        kc[i] = (s < ns) ? rows[(size_t)t * cstride + s] : 0;
    }
    for (uint32_t t = threadIdx.x; t < nt; t += blockDim.x) {
        const uint32_t mod = MODUP ? (t < level ? t : a.L + (t - level)) : t;
        mt[t] = a.mc[mod];
    }
    const uint64_t *src = a.in + b * a.in_bstride + (size_t)lo * N + c;
    uint32_t y0[MAXS], y1[MAXS];
#pragma unroll
    for (int i = 0; i < MAXS; ++i) {
        const uint64_t y = (i < (int)ns) ? src[(size_t)i * N] : 0;
        split25(y, y0[i], y1[i]);
    }
    __syncthreads();
    uint64_t *dst = a.out + b * a.out_bstride + c;
    const uint32_t per = (nt + a.tgroups - 1) / a.tgroups;
    const uint32_t t1 = min(nt, (grp + 1) * per);
#pragma unroll 2
    for (uint32_t t = grp * per; t < t1; ++t) {
        if (MODUP && t >= lo && t < lo + ns) continue;
        const ModC m = mt[t];
        const uint64_t *kr = kc + t * MAXS;
        Mac25 acc;
#pragma unroll
        for (int i = 0; i < MAXS; ++i) acc.mac(y0[i], y1[i], kr[i]);
        const uint32_t slot = MODUP ? j * ds + (t < level ? t : pbase + (t - level)) : t;
        dst[(size_t)slot * N] = acc.reduce(m.q, m.mu, m.nq);
    }
}

// Target groups of a launch: about conv_group_limbs targets per block row
// when the launch is a single step of a few ciphertexts (a thin grid: by
// default one or two ciphertexts, groups of 8), else one group.
static uint32_t conv_groups(const Ctx &c, uint32_t nt, uint32_t batch) {
    return batch <= c.plan.conv_group_max_batch ? std::max<uint32_t>(1, nt / c.plan.conv_group_limbs) : 1;
}

template <bool MODUP, bool MIXED>
static hipError_t launch_conv_m(const ConvArgs &a, uint32_t ns_max, dim3 grid, hipStream_t s) {
    if (ns_max <= 4) hipLaunchKernelGGL((conv_kernel<MODUP, 4, MIXED>), grid, dim3(256), 0, s, a);
    else if (ns_max <= 8) hipLaunchKernelGGL((conv_kernel<MODUP, 8, MIXED>), grid, dim3(256), 0, s, a);
    else if (ns_max <= 12) hipLaunchKernelGGL((conv_kernel<MODUP, 12, MIXED>), grid, dim3(256), 0, s, a);
    else if (ns_max <= 16) hipLaunchKernelGGL((conv_kernel<MODUP, 16, MIXED>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <bool MODUP>
static hipError_t launch_conv_t(const ConvArgs &a, bool mixed, uint32_t ns_max, dim3 grid, hipStream_t s) {
    return mixed ? launch_conv_m<MODUP, true>(a, ns_max, grid, s) : launch_conv_m<MODUP, false>(a, ns_max, grid, s);
}

hipError_t launch_conv_modup(const Ctx &c, const uint64_t *y, const uint32_t *levels, uint64_t *ext,
                             uint32_t batch, size_t y_bstride, size_t ext_bstride, bool keyidx, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (batch > (uint32_t)MAXB) return hipErrorInvalidValue;
    ConvArgs a{};
    a.in = y;
    a.out = ext;
    a.in_bstride = y_bstride;
    a.out_bstride = ext_bstride;
    a.conv = c.conv_modup;
    a.mc = c.mc;
    a.n = c.log_n;
    a.L = c.L;
    a.K = c.K;
    a.alpha = c.alpha;
    a.keyidx = keyidx ? 1u : 0u;
    uint32_t top = 0;
    bool mixed = false;
    for (uint32_t b = 0; b < batch; ++b) {
        if (levels[b] < 1 || levels[b] > c.L) return hipErrorInvalidValue;
        a.lvl[b] = (uint8_t)levels[b];
        a.coff[b] = (uint32_t)c.conv_modup_off[levels[b]];
        top = std::max(top, levels[b]);
        mixed = mixed || levels[b] != levels[0];
    }
    a.level0 = levels[0];
    a.coff0 = a.coff[0];
    const uint32_t beta = (top + c.alpha - 1) / c.alpha;
    a.tgroups = conv_groups(c, top + c.K, batch);
    ProfScope ps(c, HKS_K_CONV, s);
    return launch_conv_t<true>(a, mixed, c.alpha, dim3((c.n + 255) / 256, beta * a.tgroups, batch), s);
}

hipError_t launch_conv_moddown(const Ctx &c, const uint64_t *p, const uint32_t *nt, uint64_t *z, uint32_t batch,
                               size_t p_bstride, size_t z_bstride, const uint64_t *table, uint32_t ns,
                               hipStream_t s) {
    if (batch == 0) return hipSuccess;
    if (batch > (uint32_t)MAXB) return hipErrorInvalidValue;
    ConvArgs a{};
    a.in = p;
    a.out = z;
    a.conv = table;
    a.mc = c.mc;
    a.in_bstride = p_bstride;
    a.out_bstride = z_bstride;
    a.n = c.log_n;
    a.L = c.L;
    a.K = ns;      // sources: the ns special limbs
    a.alpha = c.alpha;
    uint32_t top = 0;
    bool mixed = false;
    for (uint32_t b = 0; b < batch; ++b) {
        if (nt[b] < 1 || nt[b] > c.L) return hipErrorInvalidValue;
        a.lvl[b] = (uint8_t)nt[b];  // targets q_0..q_{nt-1}
        top = std::max(top, nt[b]);
        mixed = mixed || nt[b] != nt[0];
    }
    a.level0 = nt[0];
    a.tgroups = conv_groups(c, top, batch);
    ProfScope ps(c, HKS_K_CONV, s);
    return launch_conv_t<false>(a, mixed, ns, dim3((c.n + 255) / 256, a.tgroups, batch), s);
}

// ------------------------------------------------------------------ input checks

__global__ void __launch_bounds__(256) check_kernel(const uint64_t *p, uint32_t limbs, uint32_t first_mod,
                                                    const ModC *mc, uint32_t n, uint32_t *flag) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x, limb = blockIdx.y, rep = blockIdx.z;
    if (c >= n) return;
    if (p[((size_t)rep * limbs + limb) * n + c] >= mc[first_mod + limb].q) *flag = 1u;
}

__global__ void clear_flag_kernel(uint32_t *flag) { *flag = 0u; }

hipError_t launch_check(const Ctx &c, const uint64_t *p, uint32_t reps, uint32_t limbs, uint32_t first_mod,
                        uint32_t *flag, hipStream_t s) {
    if (reps == 0 || limbs == 0) return hipSuccess;
    hipLaunchKernelGGL(check_kernel, dim3((c.n + 255) / 256, limbs, reps), dim3(256), 0, s, p, limbs, first_mod,
                       c.mc, c.n, flag);
    return hipGetLastError();
}

hipError_t launch_clear_flag(uint32_t *flag, hipStream_t s) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, s, flag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ seeded key rows

// a[j][kappa][i] for the seeded key `seed`: grid (N/256, L+K, dnum).
__global__ void __launch_bounds__(256) expand_key_a_kernel(uint64_t seed, const ModC *mc, uint64_t *a, uint32_t n,
                                                           uint32_t KL) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t kappa = blockIdx.y, j = blockIdx.z;
    if (i >= n) return;
    const ModC m = mc[kappa];
    a[((size_t)j * KL + kappa) * n + i] = seeded_key_a(seed, j, kappa, i, m.q, m.mu, m.nq);
}

hipError_t launch_expand_key_a(const Ctx &c, uint64_t seed, uint64_t *a, hipStream_t s) {
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(expand_key_a_kernel, dim3((c.n + 255) / 256, c.M, c.dnum), dim3(256), 0, s, seed, c.mc, a,
                       c.n, c.M);
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

// ------------------------------------------------------------------ encoding

// One radix-2 stage of V^H, the conjugate transpose of the special DFT
// V[j, k] = zeta^(g_j k) (zeta = exp(i pi / N), g_j = 5^j mod 2N) that maps a
// plaintext's coefficient pairs w_k = m_k + i m_(k+N/2) to its slots.
// V = S_(N/2) ... S_2 R (R the bit reversal, S_m the butterflies of block
// size m with twiddles exp(2 pi i (5^j mod 4m) / 4m)), so V^H = R S_2^H ...
// S_(N/2)^H: this kernel applies S_m^H, taking (x_r, x_(r+m/2)) to
// (x_r + x_(r+m/2), conj(w) (x_r - x_(r+m/2))) for r = b m + j, j < m/2.
__global__ void __launch_bounds__(256) enc_stage_kernel(Cplx *x, const uint32_t *rotg, const Cplx *roots,
                                                        uint32_t ns, uint32_t m) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= ns / 2) return;
    const uint32_t h = m / 2, b = tid / h, j = tid % h, r = b * m + j;
    // exp(2 pi i (5^j mod 4m) / 4m) is root (5^j mod 4m) (2N / 4m) of order 2N
    const Cplx w = roots[(rotg[j] % (4 * m)) * (ns / m)];
    const Cplx u = x[r], v = x[r + h];
    const double dr = u.re - v.re, di = u.im - v.im;
    x[r] = Cplx{u.re + v.re, u.im + v.im};
    x[r + h] = Cplx{w.re * dr + w.im * di, w.re * di - w.im * dr};
}

// The plaintext's coefficients from V^H x (bit-reversed in x): w_k =
// x[brev(k)] sc with sc = scale / (N/2); m_k = round(Re w_k) and m_(k+N/2) =
// round(Im w_k) (half to even), each reduced mod every limb of the map.
__global__ void __launch_bounds__(256) enc_round_kernel(const Cplx *x, double sc, uint32_t log_ns, const ModC *mc,
                                                        const LimbMap m, uint64_t *out, uint32_t n) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t ns = 1u << log_ns;
    if (k >= ns) return;
    const Cplx v = x[log_ns ? __brev(k) >> (32 - log_ns) : 0];
    const int64_t c[2] = {(int64_t)rint(v.re * sc), (int64_t)rint(v.im * sc)};
    for (uint32_t i = 0; i < m.count; ++i) {
        const uint64_t q = mc[m.mod[i]].q;
        uint64_t *row = out + (size_t)m.out_off[i] * n;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint64_t a = c[h] < 0 ? (uint64_t)0 - (uint64_t)c[h] : (uint64_t)c[h];
            uint64_t r = a % q;
            if (c[h] < 0 && r) r = q - r;
            row[k + h * ns] = r;
        }
    }
}

hipError_t launch_enc_fft(const Ctx &c, Cplx *x, hipStream_t s) {
    const uint32_t ns = c.n / 2;
    if (ns < 2) return hipErrorInvalidValue;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    for (uint32_t mm = ns; mm >= 2; mm /= 2)
        hipLaunchKernelGGL(enc_stage_kernel, dim3((ns / 2 + 255) / 256), dim3(256), 0, s, x, c.enc_rotg,
                           c.enc_roots, ns, mm);
    return hipGetLastError();
}

hipError_t launch_enc_round(const Ctx &c, const Cplx *x, double scale, const LimbMap &m, uint64_t *out,
                            hipStream_t s) {
    const uint32_t ns = c.n / 2;
    ProfScope ps(c, HKS_K_ELEMENTWISE, s);
    hipLaunchKernelGGL(enc_round_kernel, dim3((ns + 255) / 256), dim3(256), 0, s, x, scale / ns, c.log_n - 1, c.mc,
                       m, out, c.n);
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

// Modular-multiply throughput (hks_modmul_rate): each thread runs MR_CHAINS
// independent chains of the lazy Shoup product x <- x w mod q (values below
// 2q, the NTT butterfly's multiply) for `iters` rounds and writes one word,
// so that no product is dead code.
constexpr int MR_CHAINS = 8;

__global__ void __launch_bounds__(256) modmul_rate_kernel(uint64_t *out, uint64_t q, uint64_t nq, uint64_t w,
                                                          uint64_t wp, uint32_t iters) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t x[MR_CHAINS];
#pragma unroll
    for (int c = 0; c < MR_CHAINS; ++c) x[c] = (t * 2654435761u + 7919u * c) % q;
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < MR_CHAINS; ++c) x[c] = mul_shoup_lazy_nq(x[c], w, wp, nq);
    }
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < MR_CHAINS; ++c) acc += x[c];
    out[t] = acc;
}

hipError_t launch_modmul_rate(const Ctx &c, uint32_t iters, hipStream_t s, uint64_t *products) {
    // 32 blocks of 256 threads per CU of the 256, fewer if the workspace
    // (one word per thread) is smaller
    uint32_t blocks = 256 * 32;
    const size_t words = c.ws_bytes / sizeof(uint64_t);
    if ((size_t)blocks * 256 > words) blocks = (uint32_t)(words / 256);
    if (blocks == 0) return hipErrorInvalidValue;
    const uint64_t q = c.mods[0];
    const uint64_t w = q - 12345, wp = (uint64_t)(((unsigned __int128)w << 64) / q);
    hipLaunchKernelGGL(modmul_rate_kernel, dim3(blocks), dim3(256), 0, s, c.ws, q, 0 - q, w, wp, iters);
    *products = (uint64_t)blocks * 256 * MR_CHAINS * iters;
    return hipGetLastError();
}

hipError_t launch_copy(const uint64_t *in, uint64_t *out, size_t words, hipStream_t s) {
    if (!words) return hipSuccess;
    size_t blocks = (words + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, words);
    return hipGetLastError();
}

}  // namespace hks
