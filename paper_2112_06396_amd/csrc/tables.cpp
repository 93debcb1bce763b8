// Host-side number theory and device table construction for a context.
//   - twiddles psi^(+-brv(i)) with Shoup companions (Sec. 2.2, Sec. 2.3);
//   - ModUp conversion constants per level (Table "CKKS Subroutines",
//     Algorithm "ModUp": NewLimb over the digit's limbs);
//   - ModDown constants for dividing by P; Rescale constants (divide by the
//     last limb, round to nearest).
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "hks_internal.h"

namespace hks {

typedef unsigned __int128 u128;

uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }

uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m, b = a % m;
    for (; e; e >>= 1) {
        if (e & 1) r = h_mulmod(r, b, m);
        b = h_mulmod(b, b, m);
    }
    return r;
}

uint64_t h_invmod(uint64_t a, uint64_t m) { return h_powmod(a % m, m - 2, m); }

// Deterministic Miller-Rabin over the first twelve prime bases (exact below 2^64).
bool h_is_prime(uint64_t n) {
    const uint64_t witnesses[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t w : witnesses) {
        if (n % w == 0) return n == w;
    }
    uint64_t d = n - 1;
    unsigned r = 0;
    while (!(d & 1)) {
        d >>= 1;
        ++r;
    }
    for (uint64_t w : witnesses) {
        uint64_t x = h_powmod(w, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (unsigned i = 1; i < r && witness; ++i) {
            x = h_mulmod(x, x, n);
            if (x == n - 1) witness = false;
        }
        if (witness) return false;
    }
    return true;
}

// Primitive 2N-th root: nu^((q-1)/2N) with nu the least quadratic non-residue.
uint64_t h_root_2n(uint64_t q, uint32_t log_n) {
    uint64_t order = 2ull << log_n;
    if ((q - 1) % order) return 0;
    uint64_t nu = 2;
    while (h_powmod(nu, (q - 1) >> 1, q) != q - 1) ++nu;
    return h_powmod(nu, (q - 1) / order, q);
}

Shoup h_shoup(uint64_t w, uint64_t q) {
    Shoup s;
    s.w = w % q;
    s.wp = (uint64_t)(((u128)s.w << 64) / q);
    return s;
}

static uint32_t bitrev(uint32_t x, uint32_t bits) {
    return bits ? (__builtin_bitreverse32(x) >> (32 - bits)) : 0;
}

template <typename T>
static int upload(T **dst, const std::vector<T> &src) {
    if (src.empty()) {
        *dst = nullptr;
        return HKS_OK;
    }
    if (hipMalloc((void **)dst, sizeof(T) * src.size()) != hipSuccess) return HKS_ENOMEM;
    if (hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
        return HKS_EHIP;
    return HKS_OK;
}

// conversion constant in the split form used by the kernels: k0 | (k1 << 32),
// k = k0 + k1 2^25 with k0 < 2^25
static uint64_t split25(uint64_t k) { return (k & 0x1FFFFFFull) | ((k >> 25) << 32); }

static LastInv make_last(uint64_t q, uint64_t n_inv, uint64_t scale, uint64_t w0_inv) {
    LastInv li;
    uint64_t c = h_mulmod(n_inv, scale % q, q);
    li.c = h_shoup(c, q);
    li.cw = h_shoup(h_mulmod(c, w0_inv, q), q);
    return li;
}

int build_tables(Ctx &c) {
    const uint32_t N = c.n, M = c.M, L = c.L, K = c.K, A = c.alpha;
    std::vector<Shoup> twf((size_t)M * N), twi((size_t)M * N);
    std::vector<ModC> mc(M);
    std::vector<LastInv> lip(M);
    std::vector<uint64_t> ninv(M), w0inv(M);
    for (uint32_t m = 0; m < M; ++m) {
        uint64_t q = c.mods[m];
        uint64_t psi = h_root_2n(q, c.log_n);
        uint64_t psi_inv = h_invmod(psi, q);
        std::vector<uint64_t> pf(N), pi(N);
        pf[0] = pi[0] = 1;
        for (uint32_t e = 1; e < N; ++e) {
            pf[e] = h_mulmod(pf[e - 1], psi, q);
            pi[e] = h_mulmod(pi[e - 1], psi_inv, q);
        }
        for (uint32_t i = 0; i < N; ++i) {
            uint32_t e = bitrev(i, c.log_n);
            twf[(size_t)m * N + i] = h_shoup(pf[e], q);
            twi[(size_t)m * N + i] = h_shoup(pi[e], q);
        }
        mc[m].q = q;
        mc[m].mu = (uint64_t)(((u128)1 << 112) / q);
        mc[m].nq = 0 - q;
        {
            // -q^-1 mod 2^64 by Newton's iteration (q odd: x = q is q^-1 mod 2^3)
            uint64_t x = q;
            for (int it = 0; it < 5; ++it) x *= 2 - q * x;
            mc[m].qi = 0 - x;
        }
        ninv[m] = h_invmod(N, q);
        w0inv[m] = twi[(size_t)m * N + 1].w;
        lip[m] = make_last(q, ninv[m], 1, w0inv[m]);
    }

    // the twiddles in Montgomery form for the row passes
    std::vector<uint64_t> tmf((size_t)M * N), tmi((size_t)M * N);
    for (uint32_t m = 0; m < M; ++m) {
        const uint64_t q = c.mods[m];
        const uint64_t r64 = (uint64_t)(((u128)1 << 64) % q);  // 2^64 mod q
        for (uint32_t i = 0; i < N; ++i) {
            tmf[(size_t)m * N + i] = h_mulmod(twf[(size_t)m * N + i].w, r64, q);
            tmi[(size_t)m * N + i] = h_mulmod(twi[(size_t)m * N + i].w, r64, q);
        }
    }

    // ModUp, per level l: digit j covers [jA, min((j+1)A, l)); Qt_j over present limbs.
    std::vector<LastInv> limu((size_t)(L + 1) * L);
    c.conv_modup_off.assign(L + 1, 0);
    std::vector<uint64_t> convu;
    for (uint32_t l = 1; l <= L; ++l) {
        uint32_t beta = (l + A - 1) / A, E = l + K;
        c.conv_modup_off[l] = convu.size();
        convu.resize(convu.size() + (size_t)beta * A * E, 0);
        uint64_t *tab = convu.data() + c.conv_modup_off[l];
        for (uint32_t j = 0; j < beta; ++j) {
            uint32_t lo = j * A, hi = std::min((j + 1) * A, l);
            for (uint32_t i = lo; i < hi; ++i) {
                uint64_t qi = c.mods[i], prod = 1;
                for (uint32_t k = lo; k < hi; ++k)
                    if (k != i) prod = h_mulmod(prod, c.mods[k] % qi, qi);
                limu[(size_t)l * L + i] = make_last(qi, ninv[i], h_invmod(prod, qi), w0inv[i]);
                for (uint32_t t = 0; t < E; ++t) {
                    if (t >= lo && t < hi) continue;
                    uint64_t mt = t < l ? c.mods[t] : c.mods[L + (t - l)];
                    uint64_t v = 1;
                    for (uint32_t k = lo; k < hi; ++k)
                        if (k != i) v = h_mulmod(v, c.mods[k] % mt, mt);
                    tab[((size_t)j * E + t) * A + (i - lo)] = split25(v);
                }
            }
        }
    }

    // ModDown by P = prod p_k.
    std::vector<LastInv> limd(K);
    std::vector<uint64_t> convd((size_t)K * L);
    std::vector<Shoup> pinv(L), pmod(L);
    for (uint32_t k = 0; k < K; ++k) {
        uint64_t pk = c.mods[L + k], prod = 1;
        for (uint32_t kk = 0; kk < K; ++kk)
            if (kk != k) prod = h_mulmod(prod, c.mods[L + kk] % pk, pk);
        limd[k] = make_last(pk, ninv[L + k], h_invmod(prod, pk), w0inv[L + k]);
        for (uint32_t i = 0; i < L; ++i) {
            uint64_t qi = c.mods[i], v = 1;
            for (uint32_t kk = 0; kk < K; ++kk)
                if (kk != k) v = h_mulmod(v, c.mods[L + kk] % qi, qi);
            convd[(size_t)i * K + k] = split25(v);
        }
    }
    for (uint32_t i = 0; i < L; ++i) {
        uint64_t qi = c.mods[i], P = 1;
        for (uint32_t k = 0; k < K; ++k) P = h_mulmod(P, c.mods[L + k] % qi, qi);
        pinv[i] = h_shoup(h_invmod(P, qi), qi);
        pmod[i] = h_shoup(P, qi);
    }

    // ModDown by S = P q_{l-1} at level l (NewMult): special limbs s_0..s_{K-1} =
    // p_0..p_{K-1}, s_K = q_{l-1}; targets q_0..q_{l-2}.
    std::vector<LastInv> linm((size_t)(L + 1) * (K + 1));
    std::vector<Shoup> sinm((size_t)(L + 1) * L);
    std::vector<uint64_t> convnm;
    c.conv_nm_off.assign(L + 1, 0);
    for (uint32_t l = 2; l <= L; ++l) {
        std::vector<uint64_t> sm(K + 1);
        std::vector<uint32_t> sidx(K + 1);
        for (uint32_t k = 0; k < K; ++k) {
            sm[k] = c.mods[L + k];
            sidx[k] = L + k;
        }
        sm[K] = c.mods[l - 1];
        sidx[K] = l - 1;
        for (uint32_t k = 0; k <= K; ++k) {
            uint64_t prod = 1;
            for (uint32_t kk = 0; kk <= K; ++kk)
                if (kk != k) prod = h_mulmod(prod, sm[kk] % sm[k], sm[k]);
            linm[(size_t)l * (K + 1) + k] = make_last(sm[k], ninv[sidx[k]], h_invmod(prod, sm[k]), w0inv[sidx[k]]);
        }
        c.conv_nm_off[l] = convnm.size();
        for (uint32_t i = 0; i + 1 < l; ++i) {
            const uint64_t qi = c.mods[i];
            uint64_t all = 1;
            for (uint32_t k = 0; k <= K; ++k) {
                uint64_t v = 1;
                for (uint32_t kk = 0; kk <= K; ++kk)
                    if (kk != k) v = h_mulmod(v, sm[kk] % qi, qi);
                convnm.push_back(split25(v));
                all = h_mulmod(all, sm[k] % qi, qi);
            }
            sinm[(size_t)l * L + i] = h_shoup(h_invmod(all, qi), qi);
        }
    }

    // Rescale at level l: divide by q_{l-1}, h = (q_{l-1} - 1) / 2.
    std::vector<Shoup> rsq((size_t)(L + 1) * L);
    std::vector<uint64_t> rsh((size_t)(L + 1) * L, 0);
    for (uint32_t l = 2; l <= L; ++l) {
        uint64_t ql = c.mods[l - 1], h = (ql - 1) / 2;
        for (uint32_t i = 0; i + 1 < l; ++i) {
            uint64_t qi = c.mods[i];
            rsq[(size_t)l * L + i] = h_shoup(h_invmod(ql % qi, qi), qi);
            rsh[(size_t)l * L + i] = h % qi;
        }
    }

    // Encoding: the rotation group g_j = 5^j mod 2N (j < N/2) and the 2N-th
    // roots of unity exp(2 pi i t / 2N), rounded from long double.
    const uint32_t ns = c.n / 2, m2 = 2 * c.n;
    std::vector<uint32_t> rotg(ns);
    for (uint32_t j = 0, x = 1; j < ns; ++j, x = (uint32_t)((uint64_t)x * 5 % m2)) rotg[j] = x;
    std::vector<Cplx> roots(m2);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (uint32_t t = 0; t < m2; ++t) {
        const long double a = two_pi * (long double)t / (long double)m2;
        roots[t] = Cplx{(double)cosl(a), (double)sinl(a)};
    }

    int rc;
    if ((rc = upload(&c.enc_rotg, rotg))) return rc;
    if ((rc = upload(&c.enc_roots, roots))) return rc;
    if ((rc = upload(&c.tw_fwd, twf))) return rc;
    if ((rc = upload(&c.tw_inv, twi))) return rc;
    if ((rc = upload(&c.twm_fwd, tmf))) return rc;
    if ((rc = upload(&c.twm_inv, tmi))) return rc;
    if ((rc = upload(&c.mc, mc))) return rc;
    if ((rc = upload(&c.li_plain, lip))) return rc;
    if ((rc = upload(&c.li_modup, limu))) return rc;
    if ((rc = upload(&c.li_moddown, limd))) return rc;
    if ((rc = upload(&c.conv_modup, convu))) return rc;
    if ((rc = upload(&c.conv_moddown, convd))) return rc;
    if ((rc = upload(&c.pinv, pinv))) return rc;
    if ((rc = upload(&c.pmod, pmod))) return rc;
    if ((rc = upload(&c.li_nm, linm))) return rc;
    if ((rc = upload(&c.conv_nm, convnm))) return rc;
    if ((rc = upload(&c.sinv_nm, sinm))) return rc;
    if ((rc = upload(&c.rs_qinv, rsq))) return rc;
    if ((rc = upload(&c.rs_h, rsh))) return rc;
    return HKS_OK;
}

void free_tables(Ctx &c) {
    void *ptrs[] = {c.tw_fwd, c.tw_inv, c.twm_fwd, c.twm_inv, c.mc, c.li_plain, c.li_modup, c.li_moddown, c.conv_modup,
                    c.conv_moddown, c.pinv, c.pmod, c.rs_qinv, c.rs_h, c.ws,
                    c.li_nm, c.conv_nm, c.sinv_nm, c.enc_rotg, c.enc_roots, c.chk_flag};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    c.tw_fwd = c.tw_inv = nullptr;
    c.twm_fwd = c.twm_inv = nullptr;
    c.mc = nullptr;
    c.li_plain = c.li_modup = c.li_moddown = nullptr;
    c.conv_modup = c.conv_moddown = nullptr;
    c.pinv = c.pmod = c.rs_qinv = nullptr;
    c.li_nm = nullptr;
    c.conv_nm = nullptr;
    c.sinv_nm = nullptr;
    c.rs_h = nullptr;
    c.enc_rotg = nullptr;
    c.enc_roots = nullptr;
    c.chk_flag = nullptr;
    c.ws = nullptr;
}

}  // namespace hks
