// C ABI of the key-switching library: argument validation, context set-up,
// and the host-side orchestration of the HIP kernels for each call.
//
//   KeySwitch (Table "CKKS Subroutines"):
//     1. iNTT of the level limbs, scaled by N^-1 [(Qt_j/q_i)^-1]_{q_i}
//        (first step of ModUp, Algorithm "ModUp"); Rotate gathers the
//        automorphed input in the same kernel (Algorithm 3, line 2);
//     2. NewLimb for every digit (Decomp is a limb range of the input);
//     3. NTT of the new limbs; the digit's own limbs are copied;
//     4. KSKInnerProd against the switching key;
//     5. ModDown of u and v: iNTT of the P limbs scaled by [(P/p_k)^-1],
//        NewLimb into the q limbs, NTT, then (x - z) P^-1 (+ b_rot).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hks_internal.h"

using namespace hks;


namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? HKS_OK : HKS_EHIP; }

#define HKS_TRY(expr)                            \
    do {                                         \
        hipError_t _e = (expr);                  \
        if (_e != hipSuccess) return HKS_EHIP;   \
    } while (0)

bool aligned(const void *p) { return ((uintptr_t)p & 15u) == 0; }

uint32_t ext_mod(const Ctx &c, uint32_t level, uint32_t t) { return t < level ? t : c.L + (t - level); }

// The limbs of one call step, handed to the launchers MAXL at a time.  Fixed
// capacity (no heap use on the call path): at most beta (L + K) <= 48 * 64
// entries; an overflow makes run() fail.
struct Lists {
    static constexpr size_t CAP = 4096;
    uint16_t io[CAP], oo[CAP], ci[CAP];
    uint8_t md[CAP], dg[CAP];
    size_t size = 0;
    bool overflow = false;
    void add(uint32_t in_off, uint32_t out_off, uint32_t mod, uint32_t cidx, uint32_t digit = NO_DIGIT) {
        if (size == CAP) {
            overflow = true;
            return;
        }
        io[size] = (uint16_t)in_off;
        oo[size] = (uint16_t)out_off;
        md[size] = (uint8_t)mod;
        ci[size] = (uint16_t)cidx;
        dg[size] = (uint8_t)digit;
        ++size;
    }
    template <typename F>
    hipError_t run(F fn) const {
        if (overflow) return hipErrorInvalidValue;
        LimbMap m;
        for (size_t s = 0; s < size; s += MAXL) {
            size_t cnt = std::min<size_t>(MAXL, size - s);
            std::memset(&m, 0, sizeof(m));
            m.count = (uint32_t)cnt;
            for (size_t i = 0; i < cnt; ++i) {
                m.in_off[i] = io[s + i];
                m.out_off[i] = oo[s + i];
                m.mod[i] = md[s + i];
                m.cidx[i] = ci[s + i];
                m.dig[i] = dg[s + i];
            }
            hipError_t e = fn(m);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
};

uint32_t beta_of(const Ctx &c, uint32_t level) { return (level + c.alpha - 1) / c.alpha; }

// Canonical-range checks of call inputs (hks_set_check): `reps` copies of
// `limbs` limbs whose moduli are first_mod, first_mod + 1, ...
struct Chk {
    const uint64_t *p;
    uint32_t reps, limbs, first_mod;
};
Chk ct_chk(const uint64_t *p, uint32_t n_poly, uint32_t level) { return Chk{p, n_poly, level, 0}; }
Chk key_chk(const Ctx &c, const uint64_t *p) { return Chk{p, 2 * c.dnum, c.M, 0}; }
Chk keyb_chk(const Ctx &c, const uint64_t *p) { return Chk{p, c.dnum, c.M, 0}; }
// one polynomial over Q_level U P ([level + K][N])
void ext_chk(const Ctx &c, std::vector<Chk> &v, const uint64_t *p, uint32_t level) {
    v.push_back(Chk{p, 1, level, 0});
    v.push_back(Chk{p + (size_t)level * c.n, 1, c.K, c.L});
}

// With the context's checks on: HKS_ERANGE when a word of the items is not
// below its modulus (nothing else is enqueued then).  The check reads the
// result back and synchronizes the stream, so it refuses a capturing stream.
int check_inputs(Ctx &c, hipStream_t s, const Chk *items, size_t n_items) {
    if (!c.check) return HKS_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return HKS_EHIP;
    if (cs != hipStreamCaptureStatusNone) return HKS_EUNSUPPORTED;
    if (launch_clear_flag(c.chk_flag, s) != hipSuccess) return HKS_EHIP;
    for (size_t i = 0; i < n_items; ++i) {
        const Chk &k = items[i];
        if (k.p && launch_check(c, k.p, k.reps, k.limbs, k.first_mod, c.chk_flag, s) != hipSuccess) return HKS_EHIP;
    }
    uint32_t flag = 0;
    if (hipMemcpyAsync(&flag, c.chk_flag, sizeof(flag), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return HKS_EHIP;
    return flag ? HKS_ERANGE : HKS_OK;
}

int check_inputs(Ctx &c, hipStream_t s, const std::vector<Chk> &items) {
    return check_inputs(c, s, items.data(), items.size());
}

// (the item list is built on the stack, only when checks are on)
#define HKS_CHECKED(ctx, stream, ...)                                                             \
    do {                                                                                          \
        if ((ctx).check) {                                                                        \
            const Chk _items[] = {__VA_ARGS__};                                                   \
            const int _rc =                                                                       \
                check_inputs(ctx, (hipStream_t)(stream), _items, sizeof(_items) / sizeof(_items[0])); \
            if (_rc) return _rc;                                                                  \
        }                                                                                         \
    } while (0)

// ModUp of the converted limbs (Algorithm "ModUp") of nb polynomials at
// once, polynomial b at level levels[b]; entry b uses workspace slot b:
//   iNTT of the level limbs of a[b] (gathered through the automorph
//   galois[b]), scaled by N^-1 [(Qt_j/q_i)^-1]_{q_i} -> ws_y (coefficient form);
//   NewLimb of every digit into every other limb of Q_level U P ->
//   ext + b*ext_bstride, packed [j][t] (all levels equal) or key-indexed
//   [j][kappa] (keyidx; see launch_conv_modup);
//   forward NTT of those limbs in place (own-digit slots untouched): both
//   passes, or with cols_only just the column pass (the key-switch kernel
//   runs the row pass on chip).
int do_modup_new(Ctx &c, const Ws &w, const uint64_t *const *a, const uint32_t *galois, const uint32_t *levels,
                 uint32_t nb, uint64_t *ext, size_t ext_bstride, bool keyidx, hipStream_t s, bool cols_only) {
    const uint32_t A = c.alpha;
    uint32_t top = 0;
    bool uneven = false;
    for (uint32_t b = 0; b < nb; ++b) {
        top = std::max(top, levels[b]);
        uneven = uneven || levels[b] != levels[0];
    }
    if (uneven && !keyidx) return HKS_EINVAL;  // the packed layout is per level
    const uint32_t E = top + c.K, beta = beta_of(c, top);
    Lists inv, nl;
    // the folded scales of ModUp's iNTT are per level, at level * L + i
    // (entries at uneven levels add their own offset)
    for (uint32_t i = 0; i < top; ++i) inv.add(i, i, i, uneven ? i : top * c.L + i);
    BatchIo io{};
    for (uint32_t b = 0; b < nb; ++b) {
        io.in[b] = a[b];
        io.out[b] = w.y + b * w.st_y;
        io.galois[b] = galois[b];
        io.add_galois[b] = 1;
        if (uneven) {
            io.lvl[b] = (uint8_t)levels[b];
            io.cbase[b] = (uint16_t)(levels[b] * c.L);
        }
    }
    HKS_TRY(inv.run([&](const LimbMap &m) { return launch_ntt_inv(c, m, io, c.li_modup, nb, s); }));
    HKS_TRY(launch_conv_modup(c, w.y, levels, ext, nb, w.st_y, ext_bstride, keyidx, s));
    for (uint32_t j = 0; j < beta; ++j) {
        const uint32_t lo = j * A, hi = (j + 1) * A;
        for (uint32_t t = 0; t < E; ++t) {
            const uint32_t mod = ext_mod(c, top, t);
            if (mod < c.L && mod >= lo && mod < hi) continue;  // the digit's own limbs
            const uint32_t slot = keyidx ? j * (c.L + c.K) + mod : j * E + t;
            nl.add(slot, slot, mod, 0, j);
        }
    }
    BatchIo eio = strided_io(ext, ext_bstride, ext, ext_bstride, nb);
    for (uint32_t b = 0; b < nb && uneven; ++b) {
        eio.lvl[b] = (uint8_t)levels[b];
        eio.nbeta[b] = (uint8_t)beta_of(c, levels[b]);
    }
    HKS_TRY(nl.run([&](const LimbMap &m) {
        return cols_only ? launch_ntt_fwd_cols(c, m, eio, nb, s) : launch_ntt_fwd(c, m, eio, nb, s);
    }));
    return HKS_OK;
}

int do_modup_new(Ctx &c, const Ws &w, const uint64_t *a, uint32_t level, uint64_t *ext, hipStream_t s) {
    const uint32_t one = 1;
    return do_modup_new(c, w, &a, &one, &level, 1, ext, 0, false, s, false);
}

// The digits' own limbs of ext, copied (automorph `galois` applied) from `a`.
int do_modup_own(Ctx &c, const uint64_t *a, uint32_t level, uint32_t galois, uint64_t *ext, hipStream_t s) {
    const uint32_t A = c.alpha, E = level + c.K, beta = beta_of(c, level);
    Lists own;
    for (uint32_t j = 0; j < beta; ++j) {
        const uint32_t lo = j * A, hi = std::min((j + 1) * A, level);
        for (uint32_t t = lo; t < hi; ++t) own.add(t, j * E + t, t, 0);
    }
    HKS_TRY(own.run([&](const LimbMap &m) { return launch_automorph(c, m, a, ext, galois, 1, 1, 0, 0, s); }));
    return HKS_OK;
}

// The special limbs a ModDown divides by: the K primes of P, or for NewMult at
// level l (divide by S = P q_(l-1)) also q_(l-1), stored after them.
struct ModDownSpec {
    uint32_t ns;          // special limbs per polynomial
    uint32_t extra_mod;   // modulus index of the (K+1)-th special limb
    const LastInv *li;    // [ns] folded scales (S/s)^-1 mod s
    const uint64_t *conv; // [targets][ns] of [S/s]_{q_i}, split 25/25
    const Shoup *sinv;    // [targets] S^-1 mod q_i
};

ModDownSpec spec_by_p(const Ctx &c) { return ModDownSpec{c.K, 0, c.li_moddown, c.conv_moddown, c.pinv}; }

ModDownSpec spec_newmult(const Ctx &c, uint32_t level) {
    return ModDownSpec{c.K + 1, level - 1, c.li_nm + (size_t)level * (c.K + 1), c.conv_nm + c.conv_nm_off[level],
                       c.sinv_nm + (size_t)level * c.L};
}

// ModDown of np polynomials whose special limbs went through the inverse row
// pass into ws_p (polynomial p at ws_p + p*ns*N): inverse column pass scaled
// by N^-1 [(S/s)^-1]_s; NewLimb into the levels[p] output q limbs (ws_z +
// p*st_z); forward column pass; row pass + (u - z) S^-1 (+ add), with u, the
// output, the addend and its automorph per polynomial in `epi`.
int do_moddown_tail(Ctx &c, const Ws &w, const uint32_t *levels, uint32_t np, BatchIo epi, hipStream_t s,
                    const ModDownSpec &sp) {
    const uint32_t N = c.n, K = c.K, L = c.L;
    const size_t pst = (size_t)sp.ns * N, zst = w.st_z;
    uint32_t top = 0;
    bool uneven = false;
    for (uint32_t p = 0; p < np; ++p) {
        top = std::max(top, levels[p]);
        uneven = uneven || levels[p] != levels[0];
    }
    Lists pl, ql;
    for (uint32_t k = 0; k < K; ++k) pl.add(k, k, L + k, k);
    if (sp.ns > K) pl.add(K, K, sp.extra_mod, K);
    for (uint32_t i = 0; i < top; ++i) ql.add(i, i, i, i);
    const BatchIo pio = strided_io(w.p, pst, w.p, pst, np);
    HKS_TRY(pl.run([&](const LimbMap &m) { return launch_ntt_inv_cols(c, m, pio, sp.li, np, s); }));
    HKS_TRY(launch_conv_moddown(c, w.p, levels, w.z, np, pst, zst, sp.conv, sp.ns, s));
    BatchIo zio = strided_io(w.z, zst, w.z, zst, np);
    for (uint32_t p = 0; p < np; ++p) {
        if (uneven) {
            zio.lvl[p] = (uint8_t)levels[p];
            epi.lvl[p] = (uint8_t)levels[p];
        }
        epi.in[p] = w.z + p * zst;
    }
    HKS_TRY(ql.run([&](const LimbMap &m) { return launch_ntt_fwd_cols(c, m, zio, np, s); }));
    HKS_TRY(ql.run([&](const LimbMap &m) { return launch_rows_mdepi(c, m, epi, np, sp.sinv, s); }));
    return HKS_OK;
}

int do_moddown_tail(Ctx &c, uint32_t level, uint32_t np, BatchIo epi, hipStream_t s) {
    uint32_t levels[MAXB];
    for (uint32_t p = 0; p < np && p < (uint32_t)MAXB; ++p) levels[p] = level;
    return do_moddown_tail(c, ctx_ws(c), levels, np, epi, s, spec_by_p(c));
}

// One key-switch of a batch: d (level limbs, gathered through galois) with
// key ksk into out [2][level][N]; after ModDown, out poly 0 += add0 and
// poly 1 += add1 (each gathered through galois; null adds nothing).
struct KsJob {
    const uint64_t *d;
    uint32_t galois;
    const uint64_t *ksk;  // full key [dnum][2][L+K][N], or the rows b_j [dnum][L+K][N] of a seeded key
    uint64_t *out;
    const uint64_t *add0, *add1;
    uint32_t level = 0;
    uint64_t seed = 0;
    bool seeded = false;
    const uint64_t *newmult_bc = nullptr;  // NewMult: b3, c3 ([2][level][N]); out at level - 1
};

// KeySwitch of nb <= min(batch_cap, MAXCT) jobs in shared launches (9 per
// step); the digits' own limbs are read from d in the KSKInnerProd kernel
// (never copied), which also runs the last forward pass of ModUp's NTT.
// Jobs may sit at different levels (NewMult jobs share one): every launch
// covers the step's largest Q_level U P, and the extended digits are held
// key-indexed so that their slots do not depend on the level.
int do_keyswitch_step(Ctx &c, const Ws &w, const KsJob *jobs, uint32_t nb, hipStream_t s) {
    const uint64_t *d[MAXCT];
    uint32_t g[MAXCT], lv[MAXCT], out_lv[2 * MAXCT];
    KskBatch kb{};
    BatchIo epi{};
    // one kind per step (the entry points never mix them)
    const bool nm = jobs[0].newmult_bc != nullptr;
    for (uint32_t b = 0; b < nb; ++b) {
        const uint32_t level = jobs[b].level;
        if (level < 1 || level > c.L || (nm && level != jobs[0].level)) return HKS_EINVAL;
        const uint32_t out_level = nm ? level - 1 : level;
        d[b] = jobs[b].d;
        g[b] = jobs[b].galois;
        lv[b] = level;
        kb.direct[b] = jobs[b].d;
        kb.ksk[b] = jobs[b].ksk;
        kb.addp[b] = jobs[b].newmult_bc;
        kb.seed[b] = jobs[b].seed;
        kb.galois[b] = jobs[b].galois;
        kb.level[b] = level;
        kb.seeded = jobs[b].seeded ? 1u : 0u;
        kb.newmult = nm ? 1u : 0u;
        for (uint32_t poly = 0; poly < 2; ++poly) {
            const uint32_t p = 2 * b + poly;
            epi.uq[p] = w.uv + b * w.st_uv + poly * (size_t)level * c.n;
            epi.out[p] = jobs[b].out + poly * (size_t)out_level * c.n;
            epi.add[p] = poly ? jobs[b].add1 : jobs[b].add0;
            epi.add_galois[p] = jobs[b].galois;
            out_lv[p] = out_level;
        }
    }
    int rc = do_modup_new(c, w, d, g, lv, nb, w.ext, w.st_ext, true, s, true);
    if (rc) return rc;
    const ModDownSpec sp = nm ? spec_newmult(c, jobs[0].level) : spec_by_p(c);
    HKS_TRY(launch_ksk_rows(c, kb, nb, w.ext, w.st_ext, true, true, 0, 0, w.uv, w.st_uv, w.p,
                            (size_t)2 * sp.ns * c.n, s));
    return do_moddown_tail(c, w, out_lv, 2 * nb, epi, s, sp);
}

int do_keyswitch_jobs(Ctx &c, const KsJob *jobs, uint32_t n, hipStream_t s) {
    const uint32_t step = std::min<uint32_t>(c.batch_cap, MAXCT);
    for (uint32_t i = 0; i < n; i += step) {
        int rc = do_keyswitch_step(c, ctx_ws(c), jobs + i, std::min(step, n - i), s);
        if (rc) return rc;
    }
    return HKS_OK;
}

int do_rescale(Ctx &c, const uint64_t *ct, uint32_t level, uint64_t *out, hipStream_t s) {
    const uint32_t N = c.n;
    Lists last, rest;
    last.add(level - 1, 0, level - 1, level - 1);
    for (uint32_t i = 0; i + 1 < level; ++i) rest.add(i, i, i, 0);
    const BatchIo lio = strided_io(ct, (size_t)level * N, c.ws_r, N, 2);
    HKS_TRY(last.run([&](const LimbMap &m) { return launch_ntt_inv(c, m, lio, c.li_plain, 2, s); }));
    HKS_TRY(launch_rescale_prep(c, c.ws_r, c.ws_w, level, 2, N, (size_t)(level - 1) * N, s));
    const BatchIo wio = strided_io(c.ws_w, (size_t)(level - 1) * N, c.ws_w, (size_t)(level - 1) * N, 2);
    HKS_TRY(rest.run([&](const LimbMap &m) { return launch_ntt_fwd(c, m, wio, 2, s); }));
    HKS_TRY(launch_rescale_epi(c, ct, c.ws_w, out, level, 2, (size_t)level * N, (size_t)(level - 1) * N,
                               (size_t)(level - 1) * N, s));
    return HKS_OK;
}

bool valid_galois(const Ctx &c, uint32_t g) { return (g & 1u) && g < 2u * c.n; }

const char *status_text(int s) {
    switch (s) {
        case HKS_OK: return "ok";
        case HKS_EINVAL: return "invalid argument";
        case HKS_ENOMEM: return "out of memory";
        case HKS_EHIP: return "HIP runtime error";
        case HKS_EUNSUPPORTED: return "unsupported";
        case HKS_ERANGE: return "input residue not below its modulus";
        case HKS_ESCRATCH: return "the call needs more workspace than the allocation-free scratch holds";
        default: return "unknown status";
    }
}

}  // namespace

// ---------------------------------------------------------------- allocation-free scratch
// The workspace of hks_rotate_noalloc: a file-scope device array, one copy
// on each GPU the library runs on, held until the process ends.  In host
// code `scratch` names a host-side stand-in, not device memory: its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current, at hks_create) and only that address is handed to kernels.
static __device__ __align__(256) uint64_t scratch[HKS_NOALLOC_SCRATCH_BYTES / sizeof(uint64_t)];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
uint64_t *scratch_dev[SCRATCH_DEVICES];  // device address of `scratch` per device

// With `device` current: look up (once) the device address of its copy of
// the scratch array.  Devices beyond the table get none (the entry point
// then reports HKS_EUNSUPPORTED).
int scratch_init(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) return HKS_OK;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return HKS_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HKS_EHIP;
    scratch_dev[device] = static_cast<uint64_t *>(ptr);
    return HKS_OK;
}

uint64_t *scratch_of(int device) {
    if (device < 0 || device >= SCRATCH_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_dev[device];
}

// Words of scratch one Rotate at `level` uses: the coefficient-form input
// (level limbs), the extended digits [beta][L + K] (key-indexed slots),
// KSKInnerProd's q limbs of u and v [2][level], the special limbs of u and v
// [2][K] and ModDown's corrections [2][level].
size_t noalloc_words(const Ctx &c, uint32_t level) {
    const size_t N = c.n, beta = beta_of(c, level), M = c.M;
    return N * ((size_t)level + beta * M + 2 * (size_t)level + 2 * (size_t)c.K + 2 * (size_t)level);
}

// The workspace view of one Rotate at `level` carved from the scratch array.
Ws noalloc_ws(const Ctx &c, uint64_t *base, uint32_t level) {
    const size_t N = c.n, beta = beta_of(c, level), M = c.M;
    Ws w{};
    w.st_y = (size_t)level * N;
    w.st_ext = beta * M * N;
    w.st_uv = 2 * (size_t)level * N;
    w.st_p = 2 * (size_t)c.K * N;
    w.st_z = (size_t)level * N;  // per polynomial; u's and v's corrections
    w.y = base;
    w.ext = w.y + w.st_y;
    w.uv = w.ext + w.st_ext;
    w.p = w.uv + w.st_uv;
    w.z = w.p + w.st_p;
    return w;
}

}  // namespace

#define GUARD_BEGIN try {
#define GUARD_END                          \
    }                                      \
    catch (const std::bad_alloc &) {       \
        return HKS_ENOMEM;                 \
    }                                      \
    catch (...) {                          \
        return HKS_EINVAL;                 \
    }

extern "C" {

const char *hks_strerror(int status) { return status_text(status); }

int hks_gen_primes(uint32_t bits, uint32_t log_step, uint32_t count, uint64_t *out) {
    if (!out || bits < 8 || bits > 62 || log_step >= bits || count == 0) return HKS_EINVAL;
    const uint64_t top = 1ull << bits, step = 1ull << log_step;
    uint32_t got = 0;
    for (uint64_t k = 1; got < count; ++k) {
        if (k * step >= top) return HKS_EINVAL;
        uint64_t cand = top - k * step + 1;
        if (h_is_prime(cand)) out[got++] = cand;
    }
    return HKS_OK;
}

uint32_t hks_galois_for_rotation(int32_t k, uint32_t log_n) {
    if (log_n < 1 || log_n > 30) return 0;
    const uint64_t two_n = 2ull << log_n;
    const uint64_t slots = two_n / 4;  // 5 has order N/2 in (Z/2N)^*
    int64_t e = -(int64_t)k;           // phi_k is realized by 5^(-k)
    e %= (int64_t)slots;
    if (e < 0) e += (int64_t)slots;
    uint64_t g = 1;
    for (int64_t i = 0; i < e; ++i) g = (g * 5) % two_n;
    return (uint32_t)g;
}

uint32_t hks_galois_conjugate(uint32_t log_n) { return (uint32_t)((2ull << log_n) - 1); }

int hks_create(const hks_params *p, int device, hks_ctx **out) {
    GUARD_BEGIN
    if (!p || !out || !p->q || !p->p) return HKS_EINVAL;
    if (p->log_n < 10 || p->log_n > 16) return HKS_EINVAL;
    if (p->L < 1 || p->L > 48 || p->K < 1 || p->K > 16 || p->dnum < 1 || p->dnum > p->L) return HKS_EINVAL;
    const uint32_t alpha = (p->L + p->dnum - 1) / p->dnum;
    if (p->K < alpha || alpha > 16) return HKS_EINVAL;
    if (p->max_batch > (uint32_t)MAXCT) return HKS_EINVAL;
    std::vector<uint64_t> mods(p->q, p->q + p->L);
    mods.insert(mods.end(), p->p, p->p + p->K);
    const uint64_t two_n = 2ull << p->log_n;
    for (size_t i = 0; i < mods.size(); ++i) {
        uint64_t q = mods[i];
        if (q <= (1ull << 49) || q >= (1ull << 50) || (q - 1) % two_n || !h_is_prime(q)) return HKS_EINVAL;
        for (size_t j = 0; j < i; ++j)
            if (mods[j] == q) return HKS_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HKS_EHIP;
    if (hipSetDevice(device) != hipSuccess) return HKS_EHIP;
    if (scratch_init(device) != HKS_OK) return HKS_EHIP;
    hks_ctx *h = new hks_ctx();
    Ctx &c = h->c;
    c.device = device;
    c.log_n = p->log_n;
    c.n = 1u << p->log_n;
    c.L = p->L;
    c.K = p->K;
    c.dnum = p->dnum;
    c.alpha = alpha;
    c.M = p->L + p->K;
    c.batch_cap = p->max_batch ? p->max_batch : 1;
    c.n1 = plan_n1(c.plan, p->log_n);
    c.n2 = p->log_n - c.n1;
    c.mods = mods;
    int rc = build_tables(c);
    if (rc == HKS_OK && hipMalloc((void **)&c.chk_flag, 256) != hipSuccess) {
        c.chk_flag = nullptr;
        rc = HKS_ENOMEM;
    }
    if (const char *env = std::getenv("HKS_DEBUG_CHECK_CANONICAL")) c.check = env[0] && std::strcmp(env, "0") != 0;
    if (rc == HKS_OK) {
        const size_t N = c.n, L = c.L, cap = c.batch_cap;
        size_t words[] = {cap * c.st_y(), cap * c.st_ext(), cap * c.st_uv(), cap * c.st_p(), cap * c.st_z(),
                          cap * c.st_rot(), cap * c.st_t(), 2 * N,         2 * L * N};
        size_t total = 0;
        for (size_t w : words) total += w;
        c.ws_bytes = total * sizeof(uint64_t);
        if (hipMalloc((void **)&c.ws, c.ws_bytes) != hipSuccess) {
            c.ws = nullptr;
            rc = HKS_ENOMEM;
        } else {
            uint64_t *ptr = c.ws;
            uint64_t **slots[] = {&c.ws_y, &c.ws_ext, &c.ws_uv, &c.ws_p, &c.ws_z,
                                  &c.ws_rot, &c.ws_t, &c.ws_r, &c.ws_w};
            for (size_t i = 0; i < 9; ++i) {
                *slots[i] = ptr;
                ptr += words[i];
            }
        }
    }
    if (rc != HKS_OK) {
        free_tables(c);
        delete h;
        return rc;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        free_tables(c);
        delete h;
        return HKS_EHIP;
    }
    *out = h;
    return HKS_OK;
    GUARD_END
}

void hks_destroy(hks_ctx *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_tables(h->c);
    delete h;
}

int hks_query(const hks_ctx *h, int key, uint32_t level, uint64_t *out) {
    if (!h || !out) return HKS_EINVAL;
    const Ctx &c = h->c;
    switch (key) {
        case HKS_Q_N: *out = c.n; return HKS_OK;
        case HKS_Q_ALPHA: *out = c.alpha; return HKS_OK;
        case HKS_Q_BETA:
            if (level < 1 || level > c.L) return HKS_EINVAL;
            *out = beta_of(c, level);
            return HKS_OK;
        case HKS_Q_KSK_WORDS: *out = c.ksk_words(); return HKS_OK;
        case HKS_Q_WORKSPACE_BYTES: *out = c.ws_bytes; return HKS_OK;
        case HKS_Q_MODULUS:
            if (level >= c.M) return HKS_EINVAL;
            *out = c.mods[level];
            return HKS_OK;
        case HKS_Q_L: *out = c.L; return HKS_OK;
        case HKS_Q_K: *out = c.K; return HKS_OK;
        case HKS_Q_DNUM: *out = c.dnum; return HKS_OK;
        case HKS_Q_BATCH_CAP: *out = c.batch_cap; return HKS_OK;
        case HKS_Q_NOALLOC_BYTES:
            if (level < 1 || level > c.L) return HKS_EINVAL;
            *out = noalloc_words(c, level) * sizeof(uint64_t);
            return HKS_OK;
        case HKS_Q_NOALLOC_MAX_BYTES: *out = HKS_NOALLOC_SCRATCH_BYTES; return HKS_OK;
        default: return HKS_EINVAL;
    }
}

int hks_ntt(hks_ctx *h, uint64_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream) {
    GUARD_BEGIN
    if (!h || !x || !aligned(x) || n_limbs == 0 || first_mod + n_limbs > h->c.M) return HKS_EINVAL;
    Ctx &c = h->c;
    HKS_CHECKED(c, stream, Chk{x, 1, n_limbs, first_mod});
    Lists ls;
    for (uint32_t i = 0; i < n_limbs; ++i) ls.add(i, i, first_mod + i, first_mod + i);
    const BatchIo io = strided_io(x, 0, x, 0, 1);
    return hip_status(ls.run([&](const LimbMap &m) { return launch_ntt_fwd(c, m, io, 1, (hipStream_t)stream); }));
    GUARD_END
}

int hks_intt(hks_ctx *h, uint64_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream) {
    GUARD_BEGIN
    if (!h || !x || !aligned(x) || n_limbs == 0 || first_mod + n_limbs > h->c.M) return HKS_EINVAL;
    Ctx &c = h->c;
    HKS_CHECKED(c, stream, Chk{x, 1, n_limbs, first_mod});
    Lists ls;
    for (uint32_t i = 0; i < n_limbs; ++i) ls.add(i, i, first_mod + i, first_mod + i);
    const BatchIo io = strided_io(x, 0, x, 0, 1);
    return hip_status(
        ls.run([&](const LimbMap &m) { return launch_ntt_inv(c, m, io, c.li_plain, 1, (hipStream_t)stream); }));
    GUARD_END
}

int hks_automorph(hks_ctx *h, const uint64_t *x, uint64_t *y, uint32_t first_mod, uint32_t n_limbs,
                  uint32_t galois, int eval_domain, void *stream) {
    GUARD_BEGIN
    if (!h || !x || !y || !aligned(x) || !aligned(y) || n_limbs == 0 || first_mod + n_limbs > h->c.M)
        return HKS_EINVAL;
    Ctx &c = h->c;
    if (!valid_galois(c, galois)) return HKS_EINVAL;
    const uint64_t *xe = x + (size_t)n_limbs * c.n;
    const uint64_t *ye = y + (size_t)n_limbs * c.n;
    if (x < ye && y < xe) return HKS_EINVAL;
    HKS_CHECKED(c, stream, Chk{x, 1, n_limbs, first_mod});
    Lists ls;
    for (uint32_t i = 0; i < n_limbs; ++i) ls.add(i, i, first_mod + i, 0);
    return hip_status(ls.run([&](const LimbMap &m) {
        return launch_automorph(c, m, x, y, galois, eval_domain ? 1 : 0, 1, 0, 0, (hipStream_t)stream);
    }));
    GUARD_END
}

int hks_modup(hks_ctx *h, const uint64_t *a, uint32_t level, uint64_t *ext, void *stream) {
    GUARD_BEGIN
    if (!h || !a || !ext || !aligned(a) || !aligned(ext) || level < 1 || level > h->c.L) return HKS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HKS_CHECKED(h->c, s, ct_chk(a, 1, level));
    int rc = do_modup_new(h->c, ctx_ws(h->c), a, level, ext, s);
    return rc ? rc : do_modup_own(h->c, a, level, 1, ext, s);
    GUARD_END
}

int hks_ksk_inner(hks_ctx *h, const uint64_t *ext, uint32_t level, const uint64_t *ksk, uint64_t *uv,
                  void *stream) {
    GUARD_BEGIN
    if (!h || !ext || !ksk || !uv || !aligned(ext) || !aligned(ksk) || !aligned(uv) || level < 1 ||
        level > h->c.L)
        return HKS_EINVAL;
    Ctx &c = h->c;
    if (c.check) {
        std::vector<Chk> v{key_chk(c, ksk)};
        for (uint32_t j = 0; j < beta_of(c, level); ++j) ext_chk(c, v, ext + (size_t)j * (level + c.K) * c.n, level);
        const int rc = check_inputs(c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return hip_status(launch_ksk(c, ext, level, beta_of(c, level), ksk, uv, 1, 1, 0, 0, (hipStream_t)stream));
    GUARD_END
}

int hks_moddown(hks_ctx *h, const uint64_t *x, uint32_t level, uint64_t *y, void *stream) {
    GUARD_BEGIN
    if (!h || !x || !y || !aligned(x) || !aligned(y) || level < 1 || level > h->c.L) return HKS_EINVAL;
    Ctx &c = h->c;
    hipStream_t s = (hipStream_t)stream;
    if (c.check) {
        std::vector<Chk> v;
        ext_chk(c, v, x, level);
        const int rc = check_inputs(c, s, v);
        if (rc) return rc;
    }
    // P limbs: inverse row pass into ws_p (the column pass runs in the tail)
    Lists pl;
    for (uint32_t k = 0; k < c.K; ++k) pl.add(level + k, k, c.L + k, k);
    const BatchIo pio = strided_io(x, 0, c.ws_p, 0, 1);
    HKS_TRY(pl.run([&](const LimbMap &m) { return launch_ntt_inv_rows(c, m, pio, 1, s); }));
    BatchIo epi{};
    epi.uq[0] = x;
    epi.out[0] = y;
    epi.add_galois[0] = 1;
    return do_moddown_tail(c, level, 1, epi, s);
    GUARD_END
}

int hks_keyswitch(hks_ctx *h, const uint64_t *d, uint32_t level, const uint64_t *ksk, uint64_t *uv,
                  void *stream) {
    GUARD_BEGIN
    if (!h || !d || !ksk || !uv || !aligned(d) || !aligned(ksk) || !aligned(uv) || level < 1 ||
        level > h->c.L)
        return HKS_EINVAL;
    HKS_CHECKED(h->c, stream, ct_chk(d, 1, level), key_chk(h->c, ksk));
    const KsJob job{d, 1, ksk, uv, nullptr, nullptr, level};
    return do_keyswitch_jobs(h->c, &job, 1, (hipStream_t)stream);
    GUARD_END
}

int hks_rotate(hks_ctx *h, const uint64_t *ct, uint32_t level, uint32_t galois, const uint64_t *ksk,
               uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !ksk || !ct_out || !aligned(ct) || !aligned(ksk) || !aligned(ct_out) || level < 1 ||
        level > h->c.L || ct == ct_out)
        return HKS_EINVAL;
    Ctx &c = h->c;
    if (!valid_galois(c, galois)) return HKS_EINVAL;
    HKS_CHECKED(c, stream, ct_chk(ct, 2, level), key_chk(c, ksk));
    // (u, v + b_rot): the ModDown epilogue adds b (poly 1 of ct) gathered
    // through the automorph to v
    const KsJob job{ct, galois, ksk, ct_out, nullptr, ct + (size_t)level * c.n, level};
    return do_keyswitch_jobs(c, &job, 1, (hipStream_t)stream);
    GUARD_END
}

int hks_rotate_noalloc(hks_ctx *h, const uint64_t *ct, uint32_t level, uint32_t galois, const uint64_t *ksk,
                       uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !ksk || !ct_out || !aligned(ct) || !aligned(ksk) || !aligned(ct_out) || level < 1 ||
        level > h->c.L || ct == ct_out)
        return HKS_EINVAL;
    Ctx &c = h->c;
    if (!valid_galois(c, galois)) return HKS_EINVAL;
    if (noalloc_words(c, level) * sizeof(uint64_t) > HKS_NOALLOC_SCRATCH_BYTES) return HKS_ESCRATCH;
    uint64_t *base = scratch_of(c.device);
    if (!base) return HKS_EUNSUPPORTED;
    HKS_CHECKED(c, stream, ct_chk(ct, 2, level), key_chk(c, ksk));
    const KsJob job{ct, galois, ksk, ct_out, nullptr, ct + (size_t)level * c.n, level};
    return do_keyswitch_step(c, noalloc_ws(c, base, level), &job, 1, (hipStream_t)stream);
    GUARD_END
}

int hks_hrotate(hks_ctx *h, const uint64_t *ct, uint32_t level, uint32_t r, const uint32_t *galois,
                const uint64_t *const *ksk, uint64_t *const *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !galois || !ksk || !ct_out || !aligned(ct) || level < 1 || level > h->c.L || r == 0)
        return HKS_EINVAL;
    Ctx &c = h->c;
    for (uint32_t i = 0; i < r; ++i)
        if (!valid_galois(c, galois[i]) || !ksk[i] || !ct_out[i] || !aligned(ksk[i]) || !aligned(ct_out[i]) ||
            ct_out[i] == ct)
            return HKS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (c.check) {
        std::vector<Chk> v{ct_chk(ct, 2, level)};
        for (uint32_t i = 0; i < r; ++i) v.push_back(key_chk(c, ksk[i]));
        const int rc = check_inputs(c, s, v);
        if (rc) return rc;
    }
    const uint32_t N = c.n, E = level + c.K;
    const size_t pl = (size_t)level * N;
    int rc = do_modup_new(c, ctx_ws(c), ct, level, c.ws_ext, s);
    if (!rc) rc = do_modup_own(c, ct, level, 1, c.ws_ext, s);
    if (rc) return rc;
    // rotations in steps of up to batch_cap: one KSKInnerProd launch over the
    // shared extended digits (automorph gathered per rotation) and one ModDown
    // sequence for the step's 2 * nb polynomials
    const uint32_t step = std::min<uint32_t>(c.batch_cap, MAXCT);
    for (uint32_t i0 = 0; i0 < r; i0 += step) {
        const uint32_t nb = std::min(step, r - i0);
        KskBatch kb{};
        BatchIo epi{};
        for (uint32_t b = 0; b < nb; ++b) {
            kb.direct[b] = c.ws_ext;
            kb.ksk[b] = ksk[i0 + b];
            kb.galois[b] = galois[i0 + b];
            kb.level[b] = level;
            for (uint32_t poly = 0; poly < 2; ++poly) {
                const uint32_t p = 2 * b + poly;
                epi.uq[p] = c.ws_uv + b * c.st_uv() + poly * pl;
                epi.out[p] = ct_out[i0 + b] + poly * pl;
                epi.add[p] = poly ? ct + pl : nullptr;
                epi.add_galois[p] = galois[i0 + b];
            }
        }
        HKS_TRY(launch_ksk_rows(c, kb, nb, c.ws_ext, 0, false, false, (size_t)E * N, 1, c.ws_uv, c.st_uv(), c.ws_p,
                                (size_t)2 * c.K * N, s));
        rc = do_moddown_tail(c, level, 2 * nb, epi, s);
        if (rc) return rc;
    }
    return HKS_OK;
    GUARD_END
}

int hks_batch_rotate(hks_ctx *h, uint32_t n_ct, const uint64_t *const *ct, uint32_t level,
                     const uint32_t *galois, const uint64_t *const *ksk, uint64_t *const *ct_out,
                     void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !galois || !ksk || !ct_out || n_ct == 0 || level < 1 || level > h->c.L) return HKS_EINVAL;
    Ctx &c = h->c;
    std::vector<KsJob> jobs(n_ct);
    for (uint32_t i = 0; i < n_ct; ++i) {
        if (!ct[i] || !ksk[i] || !ct_out[i] || !aligned(ct[i]) || !aligned(ksk[i]) || !aligned(ct_out[i]) ||
            !valid_galois(c, galois[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n_ct; ++j)
            if (ct_out[i] == ct[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
        jobs[i] = KsJob{ct[i], galois[i], ksk[i], ct_out[i], nullptr, ct[i] + (size_t)level * c.n, level};
    }
    if (c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n_ct; ++i) {
            v.push_back(ct_chk(ct[i], 2, level));
            v.push_back(key_chk(c, ksk[i]));
        }
        const int rc = check_inputs(c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_keyswitch_jobs(c, jobs.data(), n_ct, (hipStream_t)stream);
    GUARD_END
}

int hks_batch_rotate_mixed(hks_ctx *h, uint32_t n_ct, const uint64_t *const *ct, const uint32_t *levels,
                           const uint32_t *galois, const uint64_t *seeds, const uint64_t *const *ksk,
                           uint64_t *const *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !levels || !galois || !ksk || !ct_out || n_ct == 0) return HKS_EINVAL;
    Ctx &c = h->c;
    std::vector<KsJob> jobs(n_ct);
    for (uint32_t i = 0; i < n_ct; ++i) {
        const uint32_t level = levels[i];
        if (level < 1 || level > c.L || !ct[i] || !ksk[i] || !ct_out[i] || !aligned(ct[i]) || !aligned(ksk[i]) ||
            !aligned(ct_out[i]) || !valid_galois(c, galois[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n_ct; ++j)
            if (ct_out[i] == ct[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
        jobs[i] = KsJob{ct[i], galois[i], ksk[i], ct_out[i], nullptr, ct[i] + (size_t)level * c.n, level,
                        seeds ? seeds[i] : 0, seeds != nullptr};
    }
    if (c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n_ct; ++i) {
            v.push_back(ct_chk(ct[i], 2, levels[i]));
            v.push_back(seeds ? keyb_chk(c, ksk[i]) : key_chk(c, ksk[i]));
        }
        const int rc = check_inputs(c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_keyswitch_jobs(c, jobs.data(), n_ct, (hipStream_t)stream);
    GUARD_END
}

int hks_ptmatvec(hks_ctx *h, const uint64_t *ct, uint32_t level, uint32_t r, const uint32_t *galois,
                 const uint64_t *const *ksk, const uint64_t *const *pt, uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !galois || !ksk || !pt || !ct_out || !aligned(ct) || !aligned(ct_out) || level < 1 ||
        level > h->c.L || r == 0 || r > (uint32_t)MAXROT || ct == ct_out)
        return HKS_EINVAL;
    Ctx &c = h->c;
    bool keyed = false;
    for (uint32_t i = 0; i < r; ++i) {
        // no key: the diagonal without rotation (galois 1)
        if (!valid_galois(c, galois[i]) || !pt[i] || !aligned(pt[i]) || (ksk[i] && !aligned(ksk[i])) ||
            (!ksk[i] && galois[i] != 1))
            return HKS_EINVAL;
        keyed = keyed || ksk[i];
    }
    hipStream_t s = (hipStream_t)stream;
    if (c.check) {
        std::vector<Chk> v{ct_chk(ct, 2, level)};
        for (uint32_t i = 0; i < r; ++i) {
            if (ksk[i]) v.push_back(key_chk(c, ksk[i]));
            ext_chk(c, v, pt[i], level);
        }
        const int rc = check_inputs(c, s, v);
        if (rc) return rc;
    }
    const size_t pl = (size_t)level * c.n;
    if (keyed) {
        int rc = do_modup_new(c, ctx_ws(c), ct, level, c.ws_ext, s);
        if (!rc) rc = do_modup_own(c, ct, level, 1, c.ws_ext, s);
        if (rc) return rc;
    }
    HKS_TRY(launch_ksk_matvec(c, c.ws_ext, level, r, galois, ksk, pt, ct, ct + pl, c.ws_uv, c.ws_p, s));
    BatchIo epi{};
    for (uint32_t p = 0; p < 2; ++p) {
        epi.uq[p] = c.ws_uv + p * pl;
        epi.out[p] = ct_out + p * pl;
        epi.add_galois[p] = 1;
    }
    return do_moddown_tail(c, level, 2, epi, s);
    GUARD_END
}

int hks_encode(hks_ctx *h, const double *slots, double scale, uint32_t level, int with_p, uint64_t *pt_out,
               void *stream) {
    GUARD_BEGIN
    if (!h || !slots || !pt_out || ((uintptr_t)slots & 15) || !aligned(pt_out) || level < 1 || level > h->c.L ||
        !(scale > 0.0) || !std::isfinite(scale))
        return HKS_EINVAL;
    Ctx &c = h->c;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t nl = level + (with_p ? c.K : 0);
    // the slots' transform runs in place in the tensor-product slot (N/2
    // complex values = N words)
    Cplx *x = reinterpret_cast<Cplx *>(c.ws_t);
    HKS_TRY(hipMemcpyAsync(x, slots, sizeof(Cplx) * (c.n / 2), hipMemcpyDeviceToDevice, s));
    HKS_TRY(launch_enc_fft(c, x, s));
    Lists ls;
    for (uint32_t i = 0; i < nl; ++i) {
        const uint32_t mod = i < level ? i : c.L + (i - level);
        ls.add(i, i, mod, mod);
    }
    HKS_TRY(ls.run([&](const LimbMap &m) { return launch_enc_round(c, x, scale, m, pt_out, s); }));
    const BatchIo io = strided_io(pt_out, 0, pt_out, 0, 1);
    return hip_status(ls.run([&](const LimbMap &m) { return launch_ntt_fwd(c, m, io, 1, s); }));
    GUARD_END
}

int hks_expand_key_a(hks_ctx *h, uint64_t seed, uint64_t *a, void *stream) {
    GUARD_BEGIN
    if (!h || !a || !aligned(a)) return HKS_EINVAL;
    return hip_status(launch_expand_key_a(h->c, seed, a, (hipStream_t)stream));
    GUARD_END
}

int hks_batch_rotate_seeded(hks_ctx *h, uint32_t n_ct, const uint64_t *const *ct, uint32_t level,
                            const uint32_t *galois, const uint64_t *seeds, const uint64_t *const *ksk_b,
                            uint64_t *const *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !galois || !seeds || !ksk_b || !ct_out || n_ct == 0 || level < 1 || level > h->c.L)
        return HKS_EINVAL;
    Ctx &c = h->c;
    std::vector<KsJob> jobs(n_ct);
    for (uint32_t i = 0; i < n_ct; ++i) {
        if (!ct[i] || !ksk_b[i] || !ct_out[i] || !aligned(ct[i]) || !aligned(ksk_b[i]) || !aligned(ct_out[i]) ||
            !valid_galois(c, galois[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n_ct; ++j)
            if (ct_out[i] == ct[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
        jobs[i] = KsJob{ct[i], galois[i], ksk_b[i], ct_out[i], nullptr, ct[i] + (size_t)level * c.n, level, seeds[i], true};
    }
    if (c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n_ct; ++i) {
            v.push_back(ct_chk(ct[i], 2, level));
            v.push_back(keyb_chk(c, ksk_b[i]));
        }
        const int rc = check_inputs(c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_keyswitch_jobs(c, jobs.data(), n_ct, (hipStream_t)stream);
    GUARD_END
}

int hks_rotate_seeded(hks_ctx *h, const uint64_t *ct, uint32_t level, uint32_t galois, uint64_t seed,
                      const uint64_t *ksk_b, uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !ksk_b || !ct_out || !aligned(ct) || !aligned(ksk_b) || !aligned(ct_out) || level < 1 ||
        level > h->c.L || ct == ct_out)
        return HKS_EINVAL;
    Ctx &c = h->c;
    if (!valid_galois(c, galois)) return HKS_EINVAL;
    HKS_CHECKED(c, stream, ct_chk(ct, 2, level), keyb_chk(c, ksk_b));
    const KsJob job{ct, galois, ksk_b, ct_out, nullptr, ct + (size_t)level * c.n, level, seed, true};
    return do_keyswitch_jobs(c, &job, 1, (hipStream_t)stream);
    GUARD_END
}

int hks_rescale(hks_ctx *h, const uint64_t *ct, uint32_t level, uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !ct_out || !aligned(ct) || !aligned(ct_out) || level < 2 || level > h->c.L || ct == ct_out)
        return HKS_EINVAL;
    HKS_CHECKED(h->c, stream, ct_chk(ct, 2, level));
    return do_rescale(h->c, ct, level, ct_out, (hipStream_t)stream);
    GUARD_END
}

int hks_ptmult(hks_ctx *h, const uint64_t *ct, const uint64_t *pt, uint32_t level, int rescale,
               uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct || !pt || !ct_out || !aligned(ct) || !aligned(pt) || !aligned(ct_out) || level < 1 ||
        level > h->c.L || (rescale && level < 2))
        return HKS_EINVAL;
    Ctx &c = h->c;
    hipStream_t s = (hipStream_t)stream;
    HKS_CHECKED(c, s, ct_chk(ct, 2, level), ct_chk(pt, 1, level));
    if (!rescale) return hip_status(launch_mulpt(c, ct, pt, ct_out, level, 2, s));
    HKS_TRY(launch_mulpt(c, ct, pt, c.ws_rot, level, 2, s));
    return do_rescale(c, c.ws_rot, level, ct_out, s);
    GUARD_END
}

// Mult (Algorithm 2) of n pairs in steps of batch_cap, pair i at level
// levels[i] (levels null: all at `level`): per pair the tensor product into
// its workspace slot, then one batched key-switch of the a1 a2 terms with the
// (b3, c3) additions, then Rescale per pair.
// (seeds non-null: rlk[i] holds only the rows b_j of seeded key seeds[i])
int do_mult_relin(Ctx &c, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2, uint32_t level,
                  const uint64_t *const *rlk, int rescale, uint64_t *const *out, hipStream_t s,
                  const uint64_t *seeds = nullptr, const uint32_t *levels = nullptr) {
    const uint32_t step = std::min<uint32_t>(c.batch_cap, MAXCT);
    for (uint32_t i0 = 0; i0 < n; i0 += step) {
        const uint32_t nb = std::min(step, n - i0);
        KsJob jobs[MAXCT];
        for (uint32_t b = 0; b < nb; ++b) {
            const uint32_t lv = levels ? levels[i0 + b] : level;
            const size_t pl = (size_t)lv * c.n;
            uint64_t *t = c.ws_t + b * c.st_t();
            HKS_TRY(launch_tensor(c, ct1[i0 + b], ct2[i0 + b], t, lv, s));
            jobs[b] = KsJob{t, 1, rlk[i0 + b], rescale ? c.ws_rot + b * c.st_rot() : out[i0 + b], t + pl, t + 2 * pl,
                            lv};
            if (seeds) {
                jobs[b].seed = seeds[i0 + b];
                jobs[b].seeded = true;
            }
        }
        int rc = do_keyswitch_step(c, ctx_ws(c), jobs, nb, s);
        if (rc) return rc;
        for (uint32_t b = 0; b < nb && rescale; ++b) {
            rc = do_rescale(c, c.ws_rot + b * c.st_rot(), jobs[b].level, out[i0 + b], s);
            if (rc) return rc;
        }
    }
    return HKS_OK;
}

// NewMult (Sec. 5.1) of n pairs at one level in steps of batch_cap: tensor
// products into the workspace slots, then one batched key-switch whose
// kernel adds P b3 / P c3 and whose ModDown divides by P q_(level-1).
int do_new_mult(Ctx &c, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2, uint32_t level,
                const uint64_t *const *rlk, uint64_t *const *out, hipStream_t s) {
    const uint32_t step = std::min<uint32_t>(c.batch_cap, MAXCT);
    for (uint32_t i0 = 0; i0 < n; i0 += step) {
        const uint32_t nb = std::min(step, n - i0);
        KsJob jobs[MAXCT];
        for (uint32_t b = 0; b < nb; ++b) {
            uint64_t *t = c.ws_t + b * c.st_t();
            HKS_TRY(launch_tensor(c, ct1[i0 + b], ct2[i0 + b], t, level, s));
            jobs[b] = KsJob{t, 1, rlk[i0 + b], out[i0 + b], nullptr, nullptr, level};
            jobs[b].newmult_bc = t + (size_t)level * c.n;
        }
        int rc = do_keyswitch_step(c, ctx_ws(c), jobs, nb, s);
        if (rc) return rc;
    }
    return HKS_OK;
}

int hks_new_mult(hks_ctx *h, const uint64_t *ct1, const uint64_t *ct2, uint32_t level, const uint64_t *rlk,
                 uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct1 || !ct2 || !rlk || !ct_out || !aligned(ct1) || !aligned(ct2) || !aligned(rlk) ||
        !aligned(ct_out) || level < 2 || level > h->c.L || ct_out == ct1 || ct_out == ct2)
        return HKS_EINVAL;
    if (h->c.K + 1 > 16) return HKS_EUNSUPPORTED;
    HKS_CHECKED(h->c, stream, ct_chk(ct1, 2, level), ct_chk(ct2, 2, level), key_chk(h->c, rlk));
    return do_new_mult(h->c, 1, &ct1, &ct2, level, &rlk, &ct_out, (hipStream_t)stream);
    GUARD_END
}

int hks_batch_new_mult(hks_ctx *h, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                       uint32_t level, const uint64_t *const *rlk, uint64_t *const *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct1 || !ct2 || !rlk || !ct_out || n == 0 || level < 2 || level > h->c.L) return HKS_EINVAL;
    if (h->c.K + 1 > 16) return HKS_EUNSUPPORTED;
    for (uint32_t i = 0; i < n; ++i) {
        if (!ct1[i] || !ct2[i] || !rlk[i] || !ct_out[i] || !aligned(ct1[i]) || !aligned(ct2[i]) ||
            !aligned(rlk[i]) || !aligned(ct_out[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n; ++j)
            if (ct_out[i] == ct1[j] || ct_out[i] == ct2[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
    }
    if (h->c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n; ++i) {
            v.push_back(ct_chk(ct1[i], 2, level));
            v.push_back(ct_chk(ct2[i], 2, level));
            v.push_back(key_chk(h->c, rlk[i]));
        }
        const int rc = check_inputs(h->c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_new_mult(h->c, n, ct1, ct2, level, rlk, ct_out, (hipStream_t)stream);
    GUARD_END
}

int hks_mult_relin(hks_ctx *h, const uint64_t *ct1, const uint64_t *ct2, uint32_t level, const uint64_t *rlk,
                   int rescale, uint64_t *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct1 || !ct2 || !rlk || !ct_out || !aligned(ct1) || !aligned(ct2) || !aligned(rlk) ||
        !aligned(ct_out) || level < 1 || level > h->c.L || (rescale && level < 2))
        return HKS_EINVAL;
    HKS_CHECKED(h->c, stream, ct_chk(ct1, 2, level), ct_chk(ct2, 2, level), key_chk(h->c, rlk));
    return do_mult_relin(h->c, 1, &ct1, &ct2, level, &rlk, rescale, &ct_out, (hipStream_t)stream);
    GUARD_END
}

int hks_batch_mult_relin(hks_ctx *h, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                         uint32_t level, const uint64_t *const *rlk, int rescale, uint64_t *const *ct_out,
                         void *stream) {
    GUARD_BEGIN
    if (!h || !ct1 || !ct2 || !rlk || !ct_out || n == 0 || level < 1 || level > h->c.L || (rescale && level < 2))
        return HKS_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        if (!ct1[i] || !ct2[i] || !rlk[i] || !ct_out[i] || !aligned(ct1[i]) || !aligned(ct2[i]) ||
            !aligned(rlk[i]) || !aligned(ct_out[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n; ++j)
            if (ct_out[i] == ct1[j] || ct_out[i] == ct2[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
    }
    if (h->c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n; ++i) {
            v.push_back(ct_chk(ct1[i], 2, level));
            v.push_back(ct_chk(ct2[i], 2, level));
            v.push_back(key_chk(h->c, rlk[i]));
        }
        const int rc = check_inputs(h->c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_mult_relin(h->c, n, ct1, ct2, level, rlk, rescale, ct_out, (hipStream_t)stream);
    GUARD_END
}

int hks_batch_mult_relin_seeded(hks_ctx *h, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                                uint32_t level, const uint64_t *seeds, const uint64_t *const *rlk_b, int rescale,
                                uint64_t *const *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct1 || !ct2 || !seeds || !rlk_b || !ct_out || n == 0 || level < 1 || level > h->c.L ||
        (rescale && level < 2))
        return HKS_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        if (!ct1[i] || !ct2[i] || !rlk_b[i] || !ct_out[i] || !aligned(ct1[i]) || !aligned(ct2[i]) ||
            !aligned(rlk_b[i]) || !aligned(ct_out[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n; ++j)
            if (ct_out[i] == ct1[j] || ct_out[i] == ct2[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
    }
    if (h->c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n; ++i) {
            v.push_back(ct_chk(ct1[i], 2, level));
            v.push_back(ct_chk(ct2[i], 2, level));
            v.push_back(keyb_chk(h->c, rlk_b[i]));
        }
        const int rc = check_inputs(h->c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_mult_relin(h->c, n, ct1, ct2, level, rlk_b, rescale, ct_out, (hipStream_t)stream, seeds);
    GUARD_END
}

int hks_batch_mult_relin_mixed(hks_ctx *h, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                               const uint32_t *levels, const uint64_t *seeds, const uint64_t *const *rlk,
                               int rescale, uint64_t *const *ct_out, void *stream) {
    GUARD_BEGIN
    if (!h || !ct1 || !ct2 || !levels || !rlk || !ct_out || n == 0) return HKS_EINVAL;
    Ctx &c = h->c;
    for (uint32_t i = 0; i < n; ++i) {
        if (levels[i] < (rescale ? 2u : 1u) || levels[i] > c.L || !ct1[i] || !ct2[i] || !rlk[i] || !ct_out[i] ||
            !aligned(ct1[i]) || !aligned(ct2[i]) || !aligned(rlk[i]) || !aligned(ct_out[i]))
            return HKS_EINVAL;
        for (uint32_t j = 0; j < n; ++j)
            if (ct_out[i] == ct1[j] || ct_out[i] == ct2[j] || (j != i && ct_out[i] == ct_out[j])) return HKS_EINVAL;
    }
    if (c.check) {
        std::vector<Chk> v;
        for (uint32_t i = 0; i < n; ++i) {
            v.push_back(ct_chk(ct1[i], 2, levels[i]));
            v.push_back(ct_chk(ct2[i], 2, levels[i]));
            v.push_back(seeds ? keyb_chk(c, rlk[i]) : key_chk(c, rlk[i]));
        }
        const int rc = check_inputs(c, (hipStream_t)stream, v);
        if (rc) return rc;
    }
    return do_mult_relin(c, n, ct1, ct2, 0, rlk, rescale, ct_out, (hipStream_t)stream, seeds, levels);
    GUARD_END
}

int hks_add(hks_ctx *h, const uint64_t *x, const uint64_t *y, uint32_t level, uint32_t n_poly, uint64_t *out,
            void *stream) {
    GUARD_BEGIN
    if (!h || !x || !y || !out || !aligned(x) || !aligned(y) || !aligned(out) || level < 1 || level > h->c.L ||
        n_poly < 1 || n_poly > 3)
        return HKS_EINVAL;
    HKS_CHECKED(h->c, stream, ct_chk(x, n_poly, level), ct_chk(y, n_poly, level));
    return hip_status(launch_add(h->c, x, y, out, n_poly * level, level, (hipStream_t)stream));
    GUARD_END
}

struct hks_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int hks_graph_begin(void *stream) {
    GUARD_BEGIN
    if (!stream) return HKS_EINVAL;  // the legacy default stream cannot be captured
    return hip_status(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    GUARD_END
}

int hks_graph_end(void *stream, hks_graph **out) {
    GUARD_BEGIN
    if (!stream || !out) return HKS_EINVAL;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture((hipStream_t)stream, &g) != hipSuccess || !g) return HKS_EHIP;
    hipGraphExec_t e = nullptr;
    if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return HKS_EHIP;
    }
    hks_graph *h = new hks_graph();
    h->graph = g;
    h->exec = e;
    *out = h;
    return HKS_OK;
    GUARD_END
}

int hks_graph_launch(hks_graph *g, void *stream) {
    GUARD_BEGIN
    if (!g || !g->exec) return HKS_EINVAL;
    return hip_status(hipGraphLaunch(g->exec, (hipStream_t)stream));
    GUARD_END
}

void hks_graph_destroy(hks_graph *g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

int hks_set_check(hks_ctx *h, int on) {
    GUARD_BEGIN
    if (!h) return HKS_EINVAL;
    h->c.check = on != 0;
    return HKS_OK;
    GUARD_END
}

int hks_get_plan(hks_ctx *h, hks_plan *out) {
    GUARD_BEGIN
    if (!h || !out) return HKS_EINVAL;
    *out = h->c.plan;
    return HKS_OK;
    GUARD_END
}

int hks_set_plan(hks_ctx *h, const hks_plan *p) {
    GUARD_BEGIN
    if (!h || !p || p->conv_group_limbs == 0 || p->conv_group_limbs > 64 || p->row_xcd_order > 1 ||
        p->ksk_xcd_order > 1 || (p->col_lines != 8 && p->col_lines != 16 && p->col_lines != 32) ||
        (p->row_lines != 4 && p->row_lines != 8 && p->row_lines != 16))
        return HKS_EINVAL;
    const uint32_t n1 = plan_n1(*p, h->c.log_n);
    if (!n1) return HKS_EINVAL;
    h->c.plan = *p;
    h->c.n1 = n1;
    h->c.n2 = h->c.log_n - n1;
    return HKS_OK;
    GUARD_END
}

int hks_prof_enable(hks_ctx *h, uint32_t mask) {
    GUARD_BEGIN
    if (!h) return HKS_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return HKS_EHIP;
    prof_reset(h->c);
    h->c.prof_mask = mask & ((1u << HKS_K_COUNT) - 1u);
    return HKS_OK;
    GUARD_END
}

int hks_modmul_rate(hks_ctx *h, uint32_t iters, void *stream, double *per_s) {
    GUARD_BEGIN
    if (!h || !per_s || iters == 0) return HKS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return HKS_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HKS_EHIP;
    }
    uint64_t products = 0;
    float ms = 0.f;
    hipError_t e = hipEventRecord(e0, s);
    if (e == hipSuccess) e = launch_modmul_rate(h->c, iters, s, &products);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return HKS_EHIP;
    *per_s = ms > 0.f ? (double)products / (ms * 1e-3) : 0.0;
    return HKS_OK;
    GUARD_END
}

int hks_prof_read(hks_ctx *h, int kernel_class, double *ms, uint64_t *launches) {
    GUARD_BEGIN
    if (!h || !ms || !launches || kernel_class < 0 || kernel_class >= HKS_K_COUNT) return HKS_EINVAL;
    const Ctx &c = h->c;
    double total = 0.0;
    for (auto &p : c.prof_ev[kernel_class]) {
        if (hipEventSynchronize(p.second) != hipSuccess) return HKS_EHIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.first, p.second) != hipSuccess) return HKS_EHIP;
        total += t;
    }
    *ms = total;
    *launches = c.prof_ev[kernel_class].size();
    return HKS_OK;
    GUARD_END
}

}  // extern "C"
