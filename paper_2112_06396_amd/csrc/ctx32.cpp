// Tables and C ABI of the 32-bit-word key-switch (include/hks32.h).  The
// number theory is the 64-bit library's host code (residues below 2^30 are
// ordinary 64-bit values there); tables are narrowed to 32-bit words.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/hks32.h"
#include "hks_internal.h"
#include "ks32.h"

namespace hks {
namespace w32 {

namespace {

typedef unsigned __int128 u128;

Shoup32 shoup32(uint64_t w, uint64_t q) {
    Shoup32 s;
    s.w = (uint32_t)(w % q);
    s.wp = (uint32_t)(((uint64_t)s.w << 32) / q);
    return s;
}

// folded last inverse stage: c = N^-1 scale, cw = c psi^-1's first twiddle
Last32 make_last32(uint64_t q, uint64_t n_inv, uint64_t scale, uint64_t w0_inv) {
    const uint64_t c = h_mulmod(n_inv, scale % q, q);
    return Last32{shoup32(c, q), shoup32(h_mulmod(c, w0_inv, q), q)};
}

uint32_t bitrev32(uint32_t x, uint32_t bits) { return bits ? (__builtin_bitreverse32(x) >> (32 - bits)) : 0; }

template <typename T>
int upload32(T **dst, const std::vector<T> &src) {
    if (src.empty()) {
        *dst = nullptr;
        return HKS_OK;
    }
    if (hipMalloc((void **)dst, sizeof(T) * src.size()) != hipSuccess) return HKS_ENOMEM;
    if (hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess) return HKS_EHIP;
    return HKS_OK;
}

}  // namespace

int build_tables32(Ctx32 &c) {
    const uint32_t N = c.n, M = c.M, L = c.L, K = c.K, A = c.alpha;
    std::vector<Shoup32> twf((size_t)M * N), twi((size_t)M * N);
    std::vector<Mod32> mc(M);
    std::vector<Last32> lip(M);
    std::vector<uint64_t> ninv(M), w0inv(M);
    for (uint32_t m = 0; m < M; ++m) {
        const uint64_t q = c.mods[m];
        const uint64_t psi = h_root_2n(q, c.log_n), psi_inv = h_invmod(psi, q);
        std::vector<uint64_t> pf(N), pi(N);
        pf[0] = pi[0] = 1;
        for (uint32_t e = 1; e < N; ++e) {
            pf[e] = h_mulmod(pf[e - 1], psi, q);
            pi[e] = h_mulmod(pi[e - 1], psi_inv, q);
        }
        for (uint32_t i = 0; i < N; ++i) {
            const uint32_t e = bitrev32(i, c.log_n);
            twf[(size_t)m * N + i] = shoup32(pf[e], q);
            twi[(size_t)m * N + i] = shoup32(pi[e], q);
        }
        mc[m].q = (uint32_t)q;
        mc[m].pad = 0;
        mc[m].mu = (uint64_t)(((u128)1 << 64) / q);
        ninv[m] = h_invmod(N, q);
        w0inv[m] = twi[(size_t)m * N + 1].w;
        lip[m] = make_last32(q, ninv[m], 1, w0inv[m]);
    }
    // ModUp per level l: digit j covers [jA, min((j+1)A, l)), Qt_j over the present limbs
    std::vector<Last32> limu((size_t)(L + 1) * L);
    c.conv_modup_off.assign(L + 1, 0);
    std::vector<uint32_t> convu;
    for (uint32_t l = 1; l <= L; ++l) {
        const uint32_t beta = (l + A - 1) / A, E = l + K;
        c.conv_modup_off[l] = convu.size();
        convu.resize(convu.size() + (size_t)beta * E * A, 0);
        uint32_t *tab = convu.data() + c.conv_modup_off[l];
        for (uint32_t j = 0; j < beta; ++j) {
            const uint32_t lo = j * A, hi = std::min((j + 1) * A, l);
            for (uint32_t i = lo; i < hi; ++i) {
                const uint64_t qi = c.mods[i];
                uint64_t prod = 1;
                for (uint32_t k = lo; k < hi; ++k)
                    if (k != i) prod = h_mulmod(prod, c.mods[k] % qi, qi);
                limu[(size_t)l * L + i] = make_last32(qi, ninv[i], h_invmod(prod, qi), w0inv[i]);
                for (uint32_t t = 0; t < E; ++t) {
                    if (t >= lo && t < hi) continue;
                    const uint64_t mt = t < l ? c.mods[t] : c.mods[L + (t - l)];
                    uint64_t v = 1;
                    for (uint32_t k = lo; k < hi; ++k)
                        if (k != i) v = h_mulmod(v, c.mods[k] % mt, mt);
                    tab[((size_t)j * E + t) * A + (i - lo)] = (uint32_t)v;
                }
            }
        }
    }
    // ModDown by P
    std::vector<Last32> limd(K);
    std::vector<uint32_t> convd((size_t)L * K);
    std::vector<Shoup32> pinv(L);
    for (uint32_t k = 0; k < K; ++k) {
        const uint64_t pk = c.mods[L + k];
        uint64_t prod = 1;
        for (uint32_t kk = 0; kk < K; ++kk)
            if (kk != k) prod = h_mulmod(prod, c.mods[L + kk] % pk, pk);
        limd[k] = make_last32(pk, ninv[L + k], h_invmod(prod, pk), w0inv[L + k]);
        for (uint32_t i = 0; i < L; ++i) {
            const uint64_t qi = c.mods[i];
            uint64_t v = 1;
            for (uint32_t kk = 0; kk < K; ++kk)
                if (kk != k) v = h_mulmod(v, c.mods[L + kk] % qi, qi);
            convd[(size_t)i * K + k] = (uint32_t)v;
        }
    }
    for (uint32_t i = 0; i < L; ++i) {
        const uint64_t qi = c.mods[i];
        uint64_t P = 1;
        for (uint32_t k = 0; k < K; ++k) P = h_mulmod(P, c.mods[L + k] % qi, qi);
        pinv[i] = shoup32(h_invmod(P, qi), qi);
    }
    int rc;
    if ((rc = upload32(&c.tw_fwd, twf))) return rc;
    if ((rc = upload32(&c.tw_inv, twi))) return rc;
    if ((rc = upload32(&c.mc, mc))) return rc;
    if ((rc = upload32(&c.li_plain, lip))) return rc;
    if ((rc = upload32(&c.li_modup, limu))) return rc;
    if ((rc = upload32(&c.li_moddown, limd))) return rc;
    if ((rc = upload32(&c.conv_modup, convu))) return rc;
    if ((rc = upload32(&c.conv_moddown, convd))) return rc;
    if ((rc = upload32(&c.pinv, pinv))) return rc;
    return HKS_OK;
}

void free_tables32(Ctx32 &c) {
    void *ptrs[] = {c.tw_fwd, c.tw_inv, c.mc, c.li_plain, c.li_modup, c.li_moddown, c.conv_modup,
                    c.conv_moddown, c.pinv, c.ws};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    c.tw_fwd = c.tw_inv = nullptr;
    c.mc = nullptr;
    c.li_plain = c.li_modup = c.li_moddown = nullptr;
    c.conv_modup = c.conv_moddown = nullptr;
    c.pinv = nullptr;
    c.ws = nullptr;
}

}  // namespace w32
}  // namespace hks

using namespace hks;
using namespace hks::w32;

struct hks32_ctx {
    Ctx32 c;
};

namespace {

int st32(hipError_t e) { return e == hipSuccess ? HKS_OK : HKS_EHIP; }
bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Map of n consecutive limbs i -> i with moduli mods[i] (first_mod + i) and
// constant index = modulus index.
Map32 consecutive(uint32_t first_mod, uint32_t n) {
    Map32 m{};
    m.count = n;
    for (uint32_t i = 0; i < n; ++i) {
        m.in_off[i] = m.out_off[i] = (uint16_t)i;
        m.mod[i] = (uint8_t)(first_mod + i);
        m.cidx[i] = (uint16_t)(first_mod + i);
    }
    return m;
}

}  // namespace

#define GUARD32_BEGIN try {
#define GUARD32_END                        \
    }                                      \
    catch (const std::bad_alloc &) {       \
        return HKS_ENOMEM;                 \
    }                                      \
    catch (...) {                          \
        return HKS_EINVAL;                 \
    }

namespace {

bool valid_galois32(const Ctx32 &c, uint32_t g) { return (g & 1) != 0 && g < 2 * c.n; }

// ModUp of automorph(a, galois) at `level` into ws_ext: inverse NTT (rows
// gathered through the automorphism, columns with (Qt_j / q_i)^-1 folded),
// NewLimb, forward column pass of the new limbs, and their row pass too when
// `full` (the digits then stay in evaluation form for several automorphisms).
hipError_t modup32(const Ctx32 &c, const uint32_t *a, uint32_t level, uint32_t galois, bool full, hipStream_t s) {
    const uint32_t A = c.alpha, K = c.K, E = level + K, beta = (level + A - 1) / A;
    Map32 inv = consecutive(0, level);
    for (uint32_t i = 0; i < level; ++i) inv.cidx[i] = (uint16_t)(level * c.L + i);
    hipError_t e = launch32_inv_rows(c, inv, a, c.ws_y, galois, s);
    if (e == hipSuccess) e = launch32_inv_cols(c, inv, c.ws_y, c.ws_y, c.li_modup, s);
    if (e == hipSuccess) e = launch32_conv_modup(c, c.ws_y, level, c.ws_ext, s);
    Map32 nl{};
    auto flush = [&]() {
        hipError_t f = launch32_fwd_cols(c, nl, c.ws_ext, c.ws_ext, s);
        if (f == hipSuccess && full) f = launch32_fwd_rows(c, nl, c.ws_ext, c.ws_ext, s);
        nl.count = 0;
        return f;
    };
    for (uint32_t j = 0; j < beta && e == hipSuccess; ++j) {
        const uint32_t lo = j * A, hi = std::min((j + 1) * A, level);
        for (uint32_t t = 0; t < E && e == hipSuccess; ++t) {
            if (t >= lo && t < hi) continue;
            if (nl.count == MAXL32) e = flush();
            const uint32_t i = nl.count++;
            nl.in_off[i] = nl.out_off[i] = (uint16_t)(j * E + t);
            nl.mod[i] = (uint8_t)(t < level ? t : c.L + (t - level));
            nl.cidx[i] = 0;
        }
    }
    if (e == hipSuccess && nl.count) e = flush();
    return e;
}

// ModDown of u and v for nrot <= HB32 key switches r (ws_uv's slot r, q
// limbs; ws_p's slot r, P limbs after their inverse row pass) into
// outs[r]: inverse column pass of the P limbs with N^-1 (P / p_k)^-1,
// NewLimb, forward NTT + (u - z) P^-1, plus b gathered through gals[r] on v.
hipError_t moddown32(const Ctx32 &c, uint32_t level, uint32_t nrot, const uint32_t *b, uint32_t *const *outs,
                     const uint32_t *gals, hipStream_t s) {
    const uint32_t K = c.K, ys = 2 * nrot;
    const size_t N = c.n;
    Map32 pm{};
    pm.count = K;
    for (uint32_t k = 0; k < K; ++k) {
        pm.in_off[k] = pm.out_off[k] = (uint16_t)k;
        pm.mod[k] = (uint8_t)(c.L + k);
        pm.cidx[k] = (uint16_t)k;
    }
    hipError_t e = launch32_inv_cols(c, pm, c.ws_p, c.ws_p, c.li_moddown, s, ys, K * N, K * N);
    if (e == hipSuccess) e = launch32_conv_moddown(c, c.ws_p, level, ys, c.ws_z, s);
    if (e == hipSuccess) {
        const Map32 zm = consecutive(0, level);
        e = launch32_fwd_cols(c, zm, c.ws_z, c.ws_z, s, ys, c.L * N, c.L * N);
    }
    if (e == hipSuccess) e = launch32_rows_epi(c, level, c.ws_z, c.ws_uv, b, nrot, outs, gals, s);
    return e;
}

}  // namespace

extern "C" {

int hks32_create(const hks32_params *p, int device, hks32_ctx **out) {
    GUARD32_BEGIN
    if (!p || !out || !p->q || !p->p) return HKS_EINVAL;
    if (p->log_n < 10 || p->log_n > 16) return HKS_EINVAL;
    if (p->L < 1 || p->L > 96 || p->K < 1 || p->K > MAXS32 || p->dnum < 1 || p->dnum > p->L) return HKS_EINVAL;
    const uint32_t alpha = (p->L + p->dnum - 1) / p->dnum;
    if (p->K < alpha || alpha > MAXS32 || p->L + p->K > MAXL32) return HKS_EINVAL;
    std::vector<uint32_t> mods(p->q, p->q + p->L);
    mods.insert(mods.end(), p->p, p->p + p->K);
    const uint64_t two_n = 2ull << p->log_n;
    for (size_t i = 0; i < mods.size(); ++i) {
        const uint64_t q = mods[i];
        if (q <= (1ull << 20) || q >= (1ull << 30) || (q - 1) % two_n || !h_is_prime(q)) return HKS_EINVAL;
        for (size_t j = 0; j < i; ++j)
            if (mods[j] == q) return HKS_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return HKS_EHIP;
    if (hipSetDevice(device) != hipSuccess) return HKS_EHIP;
    hks32_ctx *h = new hks32_ctx();
    Ctx32 &c = h->c;
    c.device = device;
    c.log_n = p->log_n;
    c.n = 1u << p->log_n;
    c.n1 = p->log_n / 2;
    c.n2 = p->log_n - c.n1;
    c.L = p->L;
    c.K = p->K;
    c.dnum = p->dnum;
    c.alpha = alpha;
    c.M = p->L + p->K;
    c.mods = mods;
    int rc = build_tables32(c);
    if (rc == HKS_OK) {
        const size_t N = c.n, L = c.L, K = c.K;
        const size_t words[] = {L * N, (size_t)c.dnum * c.M * N, HB32 * 2 * L * N, HB32 * 2 * K * N,
                                HB32 * 2 * L * N};
        size_t total = 0;
        for (size_t w : words) total += w;
        if (hipMalloc((void **)&c.ws, total * sizeof(uint32_t)) != hipSuccess) {
            c.ws = nullptr;
            rc = HKS_ENOMEM;
        } else {
            uint32_t *ptr = c.ws;
            uint32_t **slots[] = {&c.ws_y, &c.ws_ext, &c.ws_uv, &c.ws_p, &c.ws_z};
            for (size_t i = 0; i < 5; ++i) {
                *slots[i] = ptr;
                ptr += words[i];
            }
        }
    }
    if (rc == HKS_OK && hipDeviceSynchronize() != hipSuccess) rc = HKS_EHIP;
    if (rc != HKS_OK) {
        free_tables32(c);
        delete h;
        return rc;
    }
    *out = h;
    return HKS_OK;
    GUARD32_END
}

void hks32_destroy(hks32_ctx *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_tables32(h->c);
    delete h;
}

int hks32_ntt(hks32_ctx *h, uint32_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream) {
    GUARD32_BEGIN
    if (!h || !x || !al16(x) || n_limbs == 0 || first_mod + n_limbs > h->c.M) return HKS_EINVAL;
    const Ctx32 &c = h->c;
    hipStream_t s = (hipStream_t)stream;
    const Map32 m = consecutive(first_mod, n_limbs);
    hipError_t e = launch32_fwd_cols(c, m, x, x, s);
    if (e == hipSuccess) e = launch32_fwd_rows(c, m, x, x, s);
    return st32(e);
    GUARD32_END
}

int hks32_intt(hks32_ctx *h, uint32_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream) {
    GUARD32_BEGIN
    if (!h || !x || !al16(x) || n_limbs == 0 || first_mod + n_limbs > h->c.M) return HKS_EINVAL;
    const Ctx32 &c = h->c;
    hipStream_t s = (hipStream_t)stream;
    const Map32 m = consecutive(first_mod, n_limbs);
    hipError_t e = launch32_inv_rows(c, m, x, x, 1, s);
    if (e == hipSuccess) e = launch32_inv_cols(c, m, x, x, c.li_plain, s);
    return st32(e);
    GUARD32_END
}

int hks32_rotate(hks32_ctx *h, const uint32_t *ct, uint32_t level, uint32_t galois, const uint32_t *ksk,
                 uint32_t *ct_out, void *stream) {
    GUARD32_BEGIN
    if (!h || !ct || !ksk || !ct_out || !al16(ct) || !al16(ksk) || !al16(ct_out) || ct == ct_out || level < 1 ||
        level > h->c.L || !valid_galois32(h->c, galois))
        return HKS_EINVAL;
    const Ctx32 &c = h->c;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = modup32(c, ct, level, galois, false, s);
    // KSKInnerProd (+ the new limbs' row pass, + ModDown's P-limb inverse rows)
    if (e == hipSuccess) e = launch32_ksk(c, c.ws_ext, false, ct, galois, level, ksk, c.ws_uv, c.ws_p, s);
    if (e == hipSuccess) e = moddown32(c, level, 1, ct + (size_t)level * c.n, &ct_out, &galois, s);
    return st32(e);
    GUARD32_END
}

int hks32_hrotate(hks32_ctx *h, const uint32_t *ct, uint32_t level, uint32_t r, const uint32_t *galois,
                  const uint32_t *const *ksk, uint32_t *const *ct_out, void *stream) {
    GUARD32_BEGIN
    if (!h || !ct || !galois || !ksk || !ct_out || !al16(ct) || level < 1 || level > h->c.L || r == 0)
        return HKS_EINVAL;
    const Ctx32 &c = h->c;
    for (uint32_t i = 0; i < r; ++i)
        if (!valid_galois32(c, galois[i]) || !ksk[i] || !ct_out[i] || !al16(ksk[i]) || !al16(ct_out[i]) ||
            ct_out[i] == ct)
            return HKS_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // one ModUp of a, new limbs fully transformed; then per rotation the
    // KSKInnerProd gathers every digit limb through its automorphism, into
    // the rotation's slot of the workspace, and one ModDown sequence serves
    // HB32 rotations
    const size_t N = c.n;
    hipError_t e = modup32(c, ct, level, 1, true, s);
    for (uint32_t i0 = 0; i0 < r && e == hipSuccess; i0 += HB32) {
        const uint32_t nb = std::min(HB32, r - i0);
        for (uint32_t b = 0; b < nb && e == hipSuccess; ++b)
            e = launch32_ksk(c, c.ws_ext, true, ct, galois[i0 + b], level, ksk[i0 + b],
                             c.ws_uv + (size_t)b * 2 * level * N, c.ws_p + (size_t)b * 2 * c.K * N, s);
        if (e == hipSuccess) e = moddown32(c, level, nb, ct + (size_t)level * N, ct_out + i0, galois + i0, s);
    }
    return st32(e);
    GUARD32_END
}

}  // extern "C"
