/*
 * Plain CPU oracle for CKKS hybrid key-switching (de Castro et al.,
 * "Does Fully Homomorphic Encryption Need Compute Acceleration?",
 * arXiv 2112.06396).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP path.
 *
 * Style: every value is an exact residue in [0, q); every product is a
 * 128-bit integer reduced with the C '%' operator.  Loops follow the paper's
 * definitions in the order they are stated; there is no blocking, lazy
 * reduction or fusion.  Single-threaded on purpose.
 *
 * Sections of the paper followed (cited by section / table / algorithm):
 *   - RNS representation and modular arithmetic: Sec. 2.2 ("Modular
 *     Arithmetic and the Residue Number System").
 *   - Evaluation vs coefficient representation, NTT: Sec. 2.3
 *     ("Polynomial Representation").
 *   - ModDown, ModUp, Decomp, KSKInnerProd, Automorph: Table "CKKS
 *     Subroutines" and the switching-key shape of Eq. (kskShape).
 *   - ModUp as iNTT -> NewLimb -> NTT: Algorithm "ModUp" (Sec. 4.1).
 *   - PtMult, Mult, Rotate, HRotate: Algorithms 1-4 (Sec. 2.4).
 *
 * Readings where the paper is silent (kept identical in the design notes):
 *   - primes: q = 2^bits - k*2^log_step + 1, k = 1,2,..., descending, tested
 *     with deterministic Miller-Rabin (bases 2..37);
 *   - psi = nu^((q-1)/2N) with nu the smallest quadratic non-residue >= 2;
 *   - NTT(x)_j = sum_i x_i psi^(i(2 brv(j)+1)) (bit-reversed evaluation order);
 *   - digit boundaries: I_j = [j*alpha, min((j+1)*alpha, level)),
 *     alpha = ceil(L/dnum), beta = ceil(level/alpha);
 *   - ModUp is the fast basis conversion without correction;
 *   - ModDown is (U - sum_k y_k (P/p_k)) * P^-1, no rounding offset;
 *   - Rescale rounds to nearest: floor((x + (q_last-1)/2) / q_last);
 *   - switching key layout [dnum][2][L+K][N], row 0 = a_j, row 1 = b_j,
 *     key limb of q_i is i and of p_k is L+k;
 *   - decryption is a*s + b.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

typedef struct {
    uint32_t log_n;
    uint32_t L;    /* ciphertext primes at the top level */
    uint32_t K;    /* special primes (product P) */
    uint32_t dnum; /* digits in the switching key */
    const uint64_t *q; /* [L] */
    const uint64_t *p; /* [K] */
} oref_params;

/* ------------------------------------------------------------------ */
/* Scalar modular arithmetic (Sec. 2.2), written as plain definitions. */
/* ------------------------------------------------------------------ */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a * b) % m);
}
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a + b) % m);
}
static uint64_t submod(uint64_t a, uint64_t b, uint64_t m) {
    return (uint64_t)(((u128)a + m - (b % m)) % m);
}
static uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
        if (e & 1) r = mulmod(r, a, m);
        a = mulmod(a, a, m);
        e >>= 1;
    }
    return r;
}
/* m prime: Fermat inverse */
static uint64_t invmod(uint64_t a, uint64_t m) { return powmod(a % m, m - 2, m); }

uint64_t oref_mulmod(uint64_t a, uint64_t b, uint64_t m) { return mulmod(a, b, m); }
uint64_t oref_powmod(uint64_t a, uint64_t e, uint64_t m) { return powmod(a, e, m); }

/* ------------------------------------------------------------------ */
/* Primes and roots of unity                                           */
/* ------------------------------------------------------------------ */

/* Deterministic Miller-Rabin for n < 2^64 (bases 2..37). */
int oref_is_prime(uint64_t n) {
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/* count primes of the form 2^bits - k*2^log_step + 1, k = 1, 2, ... */
int oref_gen_primes(uint32_t bits, uint32_t log_step, uint32_t count, uint64_t *out) {
    if (bits < 4 || bits > 62 || log_step >= bits || count == 0) return -1;
    uint64_t top = (uint64_t)1 << bits;
    uint64_t step = (uint64_t)1 << log_step;
    uint32_t found = 0;
    for (uint64_t k = 1; found < count; k++) {
        if (k * step >= top) return -1;
        uint64_t c = top - k * step + 1;
        if (oref_is_prime(c)) out[found++] = c;
    }
    return 0;
}

/* psi = nu^((q-1)/2N), nu the smallest quadratic non-residue >= 2 (Euler). */
uint64_t oref_psi(uint64_t q, uint32_t log_n) {
    uint64_t two_n = (uint64_t)2 << log_n;
    if ((q - 1) % two_n != 0) return 0;
    uint64_t nu = 2;
    while (powmod(nu, (q - 1) / 2, q) != q - 1) nu++;
    return powmod(nu, (q - 1) / two_n, q);
}

static uint32_t brv(uint32_t x, uint32_t bits) {
    uint32_t r = 0;
    for (uint32_t i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

/* ------------------------------------------------------------------ */
/* NTT (Sec. 2.3): NTT(x)_j = sum_i x_i psi^(i (2 brv(j) + 1)) mod q.   */
/* Computed as: twist by psi^i, then the cyclic DFT with omega = psi^2 */
/* by the textbook iterative radix-2 Cooley-Tukey FFT (bit-reverse the */
/* input, then butterflies), then read the result in bit-reversed      */
/* order: NTT(x)_j = DFT(twisted)_(brv(j)).                             */
/* ------------------------------------------------------------------ */

static void cyclic_dft(uint64_t *y, uint32_t log_n, uint64_t q, uint64_t omega) {
    uint32_t n = 1u << log_n;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t r = brv(i, log_n);
        if (r > i) { uint64_t t = y[i]; y[i] = y[r]; y[r] = t; }
    }
    for (uint32_t len = 2; len <= n; len <<= 1) {
        uint64_t wlen = powmod(omega, n / len, q);
        for (uint32_t i = 0; i < n; i += len) {
            uint64_t w = 1;
            for (uint32_t k = 0; k < len / 2; k++) {
                uint64_t u = y[i + k];
                uint64_t v = mulmod(y[i + k + len / 2], w, q);
                y[i + k] = addmod(u, v, q);
                y[i + k + len / 2] = submod(u, v, q);
                w = mulmod(w, wlen, q);
            }
        }
    }
}

static void ntt_limb(uint64_t *x, uint32_t log_n, uint64_t q) {
    uint32_t n = 1u << log_n;
    uint64_t psi = oref_psi(q, log_n);
    uint64_t *y = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t pw = 1;
    for (uint32_t i = 0; i < n; i++) { y[i] = mulmod(x[i] % q, pw, q); pw = mulmod(pw, psi, q); }
    cyclic_dft(y, log_n, q, mulmod(psi, psi, q));
    for (uint32_t j = 0; j < n; j++) x[j] = y[brv(j, log_n)];
    free(y);
}

static void intt_limb(uint64_t *x, uint32_t log_n, uint64_t q) {
    uint32_t n = 1u << log_n;
    uint64_t psi = oref_psi(q, log_n);
    uint64_t psi_inv = invmod(psi, q);
    uint64_t omega_inv = mulmod(psi_inv, psi_inv, q);
    uint64_t n_inv = invmod(n, q);
    uint64_t *y = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (uint32_t k = 0; k < n; k++) y[k] = x[brv(k, log_n)] % q;
    cyclic_dft(y, log_n, q, omega_inv);
    uint64_t pw = n_inv;
    for (uint32_t i = 0; i < n; i++) { x[i] = mulmod(y[i], pw, q); pw = mulmod(pw, psi_inv, q); }
    free(y);
}

void oref_ntt(uint64_t *x, uint32_t log_n, const uint64_t *mods, uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t i = 0; i < n_limbs; i++) ntt_limb(x + i * n, log_n, mods[i]);
}

void oref_intt(uint64_t *x, uint32_t log_n, const uint64_t *mods, uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t i = 0; i < n_limbs; i++) intt_limb(x + i * n, log_n, mods[i]);
}

/* ------------------------------------------------------------------ */
/* Automorph (Table "CKKS Subroutines"): X -> X^g, g odd.              */
/* Coefficient domain: coefficient i goes to e = i*g mod 2N, negated   */
/* when e >= N.  Evaluation domain: slot j holds a(psi^(2brv(j)+1)), so */
/* the automorphed polynomial at that point is a(psi^((2brv(j)+1) g)),  */
/* which is the slot j' with 2 brv(j') + 1 = (2 brv(j) + 1) g mod 2N.   */
/* ------------------------------------------------------------------ */

void oref_automorph(const uint64_t *x, uint64_t *y, uint32_t log_n, const uint64_t *mods,
                    uint32_t n_limbs, uint32_t g, int eval_domain) {
    uint32_t n = 1u << log_n;
    uint64_t two_n = 2ull * n;
    for (uint32_t l = 0; l < n_limbs; l++) {
        const uint64_t *xi = x + (size_t)l * n;
        uint64_t *yi = y + (size_t)l * n;
        uint64_t q = mods[l];
        if (eval_domain) {
            for (uint32_t j = 0; j < n; j++) {
                uint64_t odd = ((2ull * brv(j, log_n) + 1) * g) % two_n;
                uint32_t src = brv((uint32_t)((odd - 1) / 2), log_n);
                yi[j] = xi[src];
            }
        } else {
            for (uint32_t i = 0; i < n; i++) {
                uint64_t e = ((uint64_t)i * g) % two_n;
                if (e < n) yi[e] = xi[i];
                else yi[e - n] = submod(0, xi[i], q);
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Parameter helpers                                                   */
/* ------------------------------------------------------------------ */

static uint32_t alpha_of(const oref_params *pr) { return (pr->L + pr->dnum - 1) / pr->dnum; }
static uint32_t beta_of(const oref_params *pr, uint32_t level) {
    uint32_t a = alpha_of(pr);
    return (level + a - 1) / a;
}
/* modulus of limb t of a polynomial over Q_level U P */
static uint64_t ext_mod(const oref_params *pr, uint32_t level, uint32_t t) {
    return t < level ? pr->q[t] : pr->p[t - level];
}
/* key limb index of limb t (q_i -> i, p_k -> L + k) */
static uint32_t key_limb(const oref_params *pr, uint32_t level, uint32_t t) {
    return t < level ? t : pr->L + (t - level);
}
/* The conversions keep their per-target constants in fixed arrays of
   OREF_MAX_SRC entries: at most that many limbs per digit (alpha), and at
   most OREF_MAX_SRC - 1 special primes (NewMult divides by K + 1 limbs). */
#define OREF_MAX_SRC 64
static int check(const oref_params *pr, uint32_t level) {
    if (!pr || level < 1 || level > pr->L || pr->dnum < 1 || pr->K < 1) return -1;
    if (pr->dnum > pr->L || alpha_of(pr) > OREF_MAX_SRC || pr->K + 1 > OREF_MAX_SRC) return -1;
    return 0;
}

uint32_t oref_alpha(const oref_params *pr) { return alpha_of(pr); }
uint32_t oref_beta(const oref_params *pr, uint32_t level) { return beta_of(pr, level); }

/* ------------------------------------------------------------------ */
/* ModUp (Table "CKKS Subroutines"; Algorithm "ModUp"): for each digit */
/* j of Decomp_beta, iNTT the digit's limbs, convert to every other    */
/* limb of Q_level U P with the fast basis conversion                  */
/*   xhat_t = sum_{i in I_j} [x_i (Qt/q_i)^-1]_{q_i} * (Qt/q_i)  mod t, */
/* then NTT the new limbs.  The digit's own limbs are passed through.  */
/* Output ext[j][t][N], t over q_0..q_{level-1}, p_0..p_{K-1}.          */
/* ------------------------------------------------------------------ */

int oref_modup(const oref_params *pr, const uint64_t *a, uint32_t level, uint64_t *ext) {
    if (check(pr, level)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    uint32_t alpha = alpha_of(pr), beta = beta_of(pr, level), next = level + pr->K;
    uint64_t *coef = (uint64_t *)malloc(sizeof(uint64_t) * n * level);
    memcpy(coef, a, sizeof(uint64_t) * n * level);
    oref_intt(coef, pr->log_n, pr->q, level);
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (uint32_t j = 0; j < beta; j++) {
        uint32_t lo = j * alpha, hi = (j + 1) * alpha < level ? (j + 1) * alpha : level;
        uint64_t *out = ext + (size_t)j * next * n;
        /* y_i = x_i * [(Qt/q_i)^-1]_{q_i}, in place on a copy of the digit */
        uint64_t *y = (uint64_t *)malloc(sizeof(uint64_t) * n * (hi - lo));
        for (uint32_t i = lo; i < hi; i++) {
            uint64_t qi = pr->q[i], prod = 1;
            for (uint32_t k = lo; k < hi; k++) if (k != i) prod = mulmod(prod, pr->q[k] % qi, qi);
            uint64_t inv = invmod(prod, qi);
            for (size_t c = 0; c < n; c++) y[(i - lo) * n + c] = mulmod(coef[i * n + c], inv, qi);
        }
        for (uint32_t t = 0; t < next; t++) {
            uint64_t *dst = out + (size_t)t * n;
            if (t >= lo && t < hi) { memcpy(dst, a + (size_t)t * n, sizeof(uint64_t) * n); continue; }
            uint64_t m = ext_mod(pr, level, t);
            /* constants [Qt/q_i]_t */
            uint64_t cst[OREF_MAX_SRC];
            for (uint32_t i = lo; i < hi; i++) {
                uint64_t prod = 1;
                for (uint32_t k = lo; k < hi; k++) if (k != i) prod = mulmod(prod, pr->q[k] % m, m);
                cst[i - lo] = prod;
            }
            for (size_t c = 0; c < n; c++) {
                u128 acc = 0;
                for (uint32_t i = lo; i < hi; i++) acc += (u128)y[(i - lo) * n + c] * cst[i - lo];
                tmp[c] = (uint64_t)(acc % m);
            }
            ntt_limb(tmp, pr->log_n, m);
            memcpy(dst, tmp, sizeof(uint64_t) * n);
        }
        free(y);
    }
    free(tmp);
    free(coef);
    return 0;
}

/* ------------------------------------------------------------------ */
/* KSKInnerProd (Table "CKKS Subroutines", Eq. kskShape):               */
/*   u = <ksk row 0, xhat>, v = <ksk row 1, xhat>, limb by limb.        */
/* ksk layout [dnum][2][L+K][N]; uv layout [2][level+K][N].             */
/* ------------------------------------------------------------------ */

int oref_ksk_inner(const oref_params *pr, const uint64_t *ext, uint32_t level,
                   const uint64_t *ksk, uint64_t *uv) {
    if (check(pr, level)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    uint32_t beta = beta_of(pr, level), next = level + pr->K, kl = pr->L + pr->K;
    if (beta > pr->dnum) return -1;
    for (uint32_t row = 0; row < 2; row++) {
        for (uint32_t t = 0; t < next; t++) {
            uint64_t m = ext_mod(pr, level, t);
            uint32_t kt = key_limb(pr, level, t);
            uint64_t *dst = uv + ((size_t)row * next + t) * n;
            for (size_t c = 0; c < n; c++) {
                uint64_t s = 0;
                for (uint32_t j = 0; j < beta; j++) {
                    uint64_t x = ext[((size_t)j * next + t) * n + c];
                    uint64_t k = ksk[(((size_t)j * 2 + row) * kl + kt) * n + c];
                    s = addmod(s, mulmod(x, k, m), m);
                }
                dst[c] = s;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* ModDown (Table "CKKS Subroutines"): divide by P = prod p_k and drop */
/* the K special limbs.  y_k = iNTT(x_{p_k}) * [(P/p_k)^-1]_{p_k};      */
/* z_i = NTT(sum_k y_k [P/p_k]_{q_i});  out_i = (x_i - z_i) [P^-1]_{q_i}. */
/* x: [level+K][N] eval, y: [level][N] eval.                            */
/* ------------------------------------------------------------------ */

int oref_moddown(const oref_params *pr, const uint64_t *x, uint32_t level, uint64_t *y) {
    if (check(pr, level)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    uint32_t K = pr->K;
    uint64_t *yk = (uint64_t *)malloc(sizeof(uint64_t) * n * K);
    memcpy(yk, x + (size_t)level * n, sizeof(uint64_t) * n * K);
    oref_intt(yk, pr->log_n, pr->p, K);
    for (uint32_t k = 0; k < K; k++) {
        uint64_t pk = pr->p[k], prod = 1;
        for (uint32_t kk = 0; kk < K; kk++) if (kk != k) prod = mulmod(prod, pr->p[kk] % pk, pk);
        uint64_t inv = invmod(prod, pk);
        for (size_t c = 0; c < n; c++) yk[k * n + c] = mulmod(yk[k * n + c], inv, pk);
    }
    uint64_t *z = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (uint32_t i = 0; i < level; i++) {
        uint64_t qi = pr->q[i];
        uint64_t cst[OREF_MAX_SRC];
        uint64_t pmod = 1;
        for (uint32_t k = 0; k < K; k++) {
            uint64_t prod = 1;
            for (uint32_t kk = 0; kk < K; kk++) if (kk != k) prod = mulmod(prod, pr->p[kk] % qi, qi);
            cst[k] = prod;
            pmod = mulmod(pmod, pr->p[k] % qi, qi);
        }
        uint64_t pinv = invmod(pmod, qi);
        for (size_t c = 0; c < n; c++) {
            u128 acc = 0;
            for (uint32_t k = 0; k < K; k++) acc += (u128)yk[k * n + c] * cst[k];
            z[c] = (uint64_t)(acc % qi);
        }
        ntt_limb(z, pr->log_n, qi);
        for (size_t c = 0; c < n; c++)
            y[i * n + c] = mulmod(submod(x[i * n + c], z[c], qi), pinv, qi);
    }
    free(z);
    free(yk);
    return 0;
}

/* KeySwitch = Decomp -> ModUp -> KSKInnerProd -> ModDown x2.           */
/* d: [level][N] eval; uv: [2][level][N] eval.                          */
int oref_keyswitch(const oref_params *pr, const uint64_t *d, uint32_t level,
                   const uint64_t *ksk, uint64_t *uv) {
    if (check(pr, level)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    uint32_t beta = beta_of(pr, level), next = level + pr->K;
    if (beta > pr->dnum) return -1;
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * n * next * beta);
    uint64_t *hat = (uint64_t *)malloc(sizeof(uint64_t) * n * next * 2);
    int rc = oref_modup(pr, d, level, ext);
    if (!rc) rc = oref_ksk_inner(pr, ext, level, ksk, hat);
    if (!rc) rc = oref_moddown(pr, hat, level, uv);
    if (!rc) rc = oref_moddown(pr, hat + (size_t)next * n, level, uv + (size_t)level * n);
    free(hat);
    free(ext);
    return rc;
}

/* Rotate (Algorithm 3): automorph (a, b), key-switch a_rot, add b_rot.  */
/* ct, out: [2][level][N] = (a, b) in eval form.                         */
int oref_rotate(const oref_params *pr, const uint64_t *ct, uint32_t level, uint32_t g,
                const uint64_t *ksk, uint64_t *out) {
    if (check(pr, level) || (g & 1) == 0) return -1;
    size_t n = (size_t)1 << pr->log_n;
    size_t pl = (size_t)level * n;
    uint64_t *rot = (uint64_t *)malloc(sizeof(uint64_t) * pl * 2);
    oref_automorph(ct, rot, pr->log_n, pr->q, level, g, 1);
    oref_automorph(ct + pl, rot + pl, pr->log_n, pr->q, level, g, 1);
    int rc = oref_keyswitch(pr, rot, level, ksk, out);
    if (!rc)
        for (uint32_t i = 0; i < level; i++)
            for (size_t c = 0; c < n; c++)
                out[pl + i * n + c] = addmod(out[pl + i * n + c], rot[pl + i * n + c], pr->q[i]);
    free(rot);
    return rc;
}

/* HRotate (Algorithm 4): ModUp once; per rotation automorph the       */
/* extended digits, KSKInnerProd, ModDown x2, add automorphed b.        */
int oref_hrotate(const oref_params *pr, const uint64_t *ct, uint32_t level, uint32_t r,
                 const uint32_t *gs, const uint64_t *const *ksks, uint64_t *const *outs) {
    if (check(pr, level)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    size_t pl = (size_t)level * n;
    uint32_t beta = beta_of(pr, level), next = level + pr->K;
    if (beta > pr->dnum) return -1;
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * n * next * beta);
    uint64_t *erot = (uint64_t *)malloc(sizeof(uint64_t) * n * next * beta);
    uint64_t *hat = (uint64_t *)malloc(sizeof(uint64_t) * n * next * 2);
    uint64_t *brot = (uint64_t *)malloc(sizeof(uint64_t) * pl);
    uint64_t *emods = (uint64_t *)malloc(sizeof(uint64_t) * next);
    for (uint32_t t = 0; t < next; t++) emods[t] = ext_mod(pr, level, t);
    int rc = oref_modup(pr, ct, level, ext);
    for (uint32_t i = 0; !rc && i < r; i++) {
        if ((gs[i] & 1) == 0) { rc = -1; break; }
        for (uint32_t j = 0; j < beta; j++)
            oref_automorph(ext + (size_t)j * next * n, erot + (size_t)j * next * n, pr->log_n,
                           emods, next, gs[i], 1);
        rc = oref_ksk_inner(pr, erot, level, ksks[i], hat);
        if (!rc) rc = oref_moddown(pr, hat, level, outs[i]);
        if (!rc) rc = oref_moddown(pr, hat + (size_t)next * n, level, outs[i] + pl);
        if (rc) break;
        oref_automorph(ct + pl, brot, pr->log_n, pr->q, level, gs[i], 1);
        for (uint32_t l = 0; l < level; l++)
            for (size_t c = 0; c < n; c++)
                outs[i][pl + l * n + c] = addmod(outs[i][pl + l * n + c], brot[l * n + c], pr->q[l]);
    }
    free(emods);
    free(brot);
    free(hat);
    free(erot);
    free(ext);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Rescale = ModDown_{B,1} (Sec. 2.4, "Handling a Growing Scaling      */
/* Factor"): divide by the last limb q_last and round to nearest.       */
/* With h = (q_last - 1)/2 and r = (x + h) mod q_last (coefficient      */
/* form), out_i = (x_i + h - r) * q_last^-1 mod q_i.                    */
/* poly: [level][N] eval -> [level-1][N] eval.                          */
/* ------------------------------------------------------------------ */

static void rescale_poly(const oref_params *pr, const uint64_t *x, uint32_t level, uint64_t *y) {
    size_t n = (size_t)1 << pr->log_n;
    uint64_t ql = pr->q[level - 1], h = (ql - 1) / 2;
    uint64_t *r = (uint64_t *)malloc(sizeof(uint64_t) * n);
    uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * n);
    memcpy(r, x + (size_t)(level - 1) * n, sizeof(uint64_t) * n);
    intt_limb(r, pr->log_n, ql);
    for (size_t c = 0; c < n; c++) r[c] = addmod(r[c], h, ql);
    for (uint32_t i = 0; i + 1 < level; i++) {
        uint64_t qi = pr->q[i];
        for (size_t c = 0; c < n; c++) w[c] = submod(r[c] % qi, h % qi, qi);
        ntt_limb(w, pr->log_n, qi);
        uint64_t inv = invmod(ql % qi, qi);
        for (size_t c = 0; c < n; c++) y[i * n + c] = mulmod(submod(x[i * n + c], w[c], qi), inv, qi);
    }
    free(w);
    free(r);
}

int oref_rescale(const oref_params *pr, const uint64_t *ct, uint32_t level, uint64_t *out) {
    if (check(pr, level) || level < 2) return -1;
    size_t n = (size_t)1 << pr->log_n;
    rescale_poly(pr, ct, level, out);
    rescale_poly(pr, ct + (size_t)level * n, level, out + (size_t)(level - 1) * n);
    return 0;
}

/* PtMult (Algorithm 1): (a*pt, b*pt), then Rescale when asked.          */
int oref_ptmult(const oref_params *pr, const uint64_t *ct, const uint64_t *pt, uint32_t level,
                int rescale, uint64_t *out) {
    if (check(pr, level) || (rescale && level < 2)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    size_t pl = (size_t)level * n;
    uint64_t *t = (uint64_t *)malloc(sizeof(uint64_t) * pl * 2);
    for (uint32_t poly = 0; poly < 2; poly++)
        for (uint32_t i = 0; i < level; i++)
            for (size_t c = 0; c < n; c++)
                t[poly * pl + i * n + c] = mulmod(ct[poly * pl + i * n + c], pt[i * n + c], pr->q[i]);
    if (rescale) oref_rescale(pr, t, level, out);
    else memcpy(out, t, sizeof(uint64_t) * pl * 2);
    free(t);
    return 0;
}

/* Mult (Algorithm 2): tensor, key-switch a3 with the relinearization   */
/* key, (b3 + u, c3 + v), then Rescale when asked.                       */
int oref_mult_relin(const oref_params *pr, const uint64_t *ct1, const uint64_t *ct2,
                    uint32_t level, const uint64_t *rlk, int rescale, uint64_t *out) {
    if (check(pr, level) || (rescale && level < 2)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    size_t pl = (size_t)level * n;
    uint64_t *a3 = (uint64_t *)malloc(sizeof(uint64_t) * pl);
    uint64_t *bc = (uint64_t *)malloc(sizeof(uint64_t) * pl * 2);
    uint64_t *uv = (uint64_t *)malloc(sizeof(uint64_t) * pl * 2);
    for (uint32_t i = 0; i < level; i++) {
        uint64_t q = pr->q[i];
        for (size_t c = 0; c < n; c++) {
            size_t o = i * n + c;
            uint64_t a1 = ct1[o], b1 = ct1[pl + o], a2 = ct2[o], b2 = ct2[pl + o];
            a3[o] = mulmod(a1, a2, q);
            bc[o] = addmod(mulmod(a1, b2, q), mulmod(a2, b1, q), q);
            bc[pl + o] = mulmod(b1, b2, q);
        }
    }
    int rc = oref_keyswitch(pr, a3, level, rlk, uv);
    if (!rc) {
        for (uint32_t i = 0; i < level; i++)
            for (size_t c = 0; c < n; c++) {
                size_t o = i * n + c;
                uv[o] = addmod(bc[o], uv[o], pr->q[i]);
                uv[pl + o] = addmod(bc[pl + o], uv[pl + o], pr->q[i]);
            }
        if (rescale) rc = oref_rescale(pr, uv, level, out);
        else memcpy(out, uv, sizeof(uint64_t) * pl * 2);
    }
    free(uv);
    free(bc);
    free(a3);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Limb-wise helpers used by key generation and encryption in tests.   */
/* ------------------------------------------------------------------ */

void oref_mul_vec(const uint64_t *x, const uint64_t *y, uint64_t *out, uint32_t log_n,
                  const uint64_t *mods, uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t l = 0; l < n_limbs; l++)
        for (size_t c = 0; c < n; c++) out[l * n + c] = mulmod(x[l * n + c], y[l * n + c], mods[l]);
}
void oref_add_vec(const uint64_t *x, const uint64_t *y, uint64_t *out, uint32_t log_n,
                  const uint64_t *mods, uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t l = 0; l < n_limbs; l++)
        for (size_t c = 0; c < n; c++) out[l * n + c] = addmod(x[l * n + c], y[l * n + c], mods[l]);
}
void oref_sub_vec(const uint64_t *x, const uint64_t *y, uint64_t *out, uint32_t log_n,
                  const uint64_t *mods, uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t l = 0; l < n_limbs; l++)
        for (size_t c = 0; c < n; c++) out[l * n + c] = submod(x[l * n + c], y[l * n + c], mods[l]);
}
void oref_scale_vec(const uint64_t *x, const uint64_t *scalars, uint64_t *out, uint32_t log_n,
                    const uint64_t *mods, uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t l = 0; l < n_limbs; l++)
        for (size_t c = 0; c < n; c++) out[l * n + c] = mulmod(x[l * n + c], scalars[l] % mods[l], mods[l]);
}
/* residues of a signed integer polynomial: out[l][c] = v[c] mod mods[l] */
void oref_lift_signed(const int64_t *v, uint64_t *out, uint32_t log_n, const uint64_t *mods,
                      uint32_t n_limbs) {
    size_t n = (size_t)1 << log_n;
    for (uint32_t l = 0; l < n_limbs; l++)
        for (size_t c = 0; c < n; c++) {
            int64_t s = v[c];
            uint64_t m = mods[l];
            uint64_t r = s >= 0 ? ((uint64_t)s) % m : (m - ((uint64_t)(-(s + 1)) + 1) % m) % m;
            out[l * n + c] = r;
        }
}

/* ---------------------------------------------------------------------------
 * Seeded switching keys (the paper's key compression, Sec. 5.3: the uniform
 * row a_j of a switching key is regenerated from a short seed instead of
 * being stored).  The generator is Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3", SC 2011), written
 * here from its published definition: ten rounds of
 *   (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
 * with M0 = 0xD2511F53, M1 = 0xCD9E8D57, the key (k0, k1) advanced by
 * (0x9E3779B9, 0xBB67AE85) before every round after the first.
 * ------------------------------------------------------------------------- */
void oref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* The uniform rows of a seeded key, [dnum][L+K][N]: entry (j, kappa, i), for
 * key limb kappa (q_kappa for kappa < L, p_(kappa-L) after), is the 96-bit
 * number c0 + c1 2^32 + c2 2^64 reduced mod that limb's prime, where
 * (c0, c1, c2, c3) = Philox4x32-10(counter (i, kappa, j, 0x4B53),
 * key (seed mod 2^32, seed >> 32)).  (Reduction bias below 2^-46.) */
void oref_expand_key_a(const oref_params *pr, uint64_t seed, uint64_t *a) {
    const uint32_t n = 1u << pr->log_n, KL = pr->L + pr->K;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t j = 0; j < pr->dnum; ++j)
        for (uint32_t kappa = 0; kappa < KL; ++kappa) {
            const uint64_t m = kappa < pr->L ? pr->q[kappa] : pr->p[kappa - pr->L];
            for (uint32_t i = 0; i < n; ++i) {
                const uint32_t ctr[4] = {i, kappa, j, 0x4B53u};
                uint32_t o[4];
                oref_philox4x32_10(ctr, key, o);
                const u128 y = ((u128)o[2] << 64) | ((u128)o[1] << 32) | o[0];
                a[((size_t)j * KL + kappa) * n + i] = (uint64_t)(y % m);
            }
        }
}

/* ---------------------------------------------------------------------------
 * PtMatVecMult with the ModDown hoisted out of the rotation loop (Sec. 5.2,
 * Algorithm "PtMatVecMult"): sum_i M_i * Rotate_{g_i}(x) with one ModDown.
 *   ModUp of a_x once; for each i: automorph the extended digits by g_i,
 *   KSKInnerProd with ksk_i -> (u, v) over Q_level U P; b_rot = automorph of
 *   b_x; PModUp(b_rot) = P * b_rot on the q limbs, 0 on the P limbs;
 *   accumulate (a_y, b_y) += M_i * (u, v + PModUp(b_rot)) limb-wise; finally
 *   out = (ModDown(a_y), ModDown(b_y)).
 * pts[i] is the diagonal M_i given over the extended basis ([level + K][N],
 * evaluation form, residues mod q_0..q_{level-1}, p_0..p_{K-1}): the
 * plaintext itself, not multiplied by P (a factor P on it would survive the
 * single ModDown).  ksks[i] == NULL with g_i = 1 is the diagonal without a
 * rotation (offset 0 of a factored DFT matrix): its (u, v) is PModUp of the
 * input, (P a, P b) on the q limbs, with no key switch; since ModDown is
 * exact on multiples of P, that term alone gives M_0 * (a, b).
 * ------------------------------------------------------------------------- */
int oref_ptmatvec(const oref_params *pr, const uint64_t *ct, uint32_t level, uint32_t r, const uint32_t *gs,
                  const uint64_t *const *ksks, const uint64_t *const *pts, uint64_t *out) {
    if (check(pr, level)) return -1;
    size_t n = (size_t)1 << pr->log_n;
    size_t pl = (size_t)level * n;
    uint32_t beta = beta_of(pr, level), next = level + pr->K;
    if (beta > pr->dnum) return -1;
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * n * next * beta);
    uint64_t *erot = (uint64_t *)malloc(sizeof(uint64_t) * n * next * beta);
    uint64_t *hat = (uint64_t *)malloc(sizeof(uint64_t) * n * next * 2);
    uint64_t *acc = (uint64_t *)calloc(n * next * 2, sizeof(uint64_t));
    uint64_t *brot = (uint64_t *)malloc(sizeof(uint64_t) * pl);
    uint64_t *emods = (uint64_t *)malloc(sizeof(uint64_t) * next);
    for (uint32_t t = 0; t < next; t++) emods[t] = ext_mod(pr, level, t);
    int rc = oref_modup(pr, ct, level, ext);
    for (uint32_t i = 0; !rc && i < r; i++) {
        if ((gs[i] & 1) == 0) { rc = -1; break; }
        if (ksks[i] == NULL) {
            /* the diagonal without rotation: (u, v) = (PModUp(a), 0), no key
               switch (P a on the q limbs, 0 on the P limbs) */
            if (gs[i] != 1) { rc = -1; break; }
            for (uint32_t t = 0; t < next; t++) {
                uint64_t m = emods[t], pmod = 1;
                for (uint32_t k = 0; k < pr->K; k++) pmod = mulmod(pmod, pr->p[k] % m, m);
                for (size_t c = 0; c < n; c++) {
                    hat[t * n + c] = t < level ? mulmod(pmod, ct[t * n + c], m) : 0;
                    hat[((size_t)next + t) * n + c] = 0;
                }
            }
        } else {
            for (uint32_t j = 0; j < beta; j++)
                oref_automorph(ext + (size_t)j * next * n, erot + (size_t)j * next * n, pr->log_n,
                               emods, next, gs[i], 1);
            rc = oref_ksk_inner(pr, erot, level, ksks[i], hat);
            if (rc) break;
        }
        oref_automorph(ct + pl, brot, pr->log_n, pr->q, level, gs[i], 1);
        for (uint32_t t = 0; t < next; t++) {
            uint64_t m = emods[t];
            uint64_t pmod = 1;  /* [P]_m on q limbs; PModUp is 0 on the P limbs */
            for (uint32_t k = 0; k < pr->K; k++) pmod = mulmod(pmod, pr->p[k] % m, m);
            for (size_t c = 0; c < n; c++) {
                uint64_t mi = pts[i][t * n + c];
                uint64_t u = hat[t * n + c], v = hat[((size_t)next + t) * n + c];
                uint64_t bh = t < level ? mulmod(pmod, brot[t * n + c], m) : 0;
                acc[t * n + c] = addmod(acc[t * n + c], mulmod(mi, u, m), m);
                acc[((size_t)next + t) * n + c] = addmod(acc[((size_t)next + t) * n + c],
                                                         mulmod(mi, addmod(v, bh, m), m), m);
            }
        }
    }
    if (!rc) rc = oref_moddown(pr, acc, level, out);
    if (!rc) rc = oref_moddown(pr, acc + (size_t)next * n, level, out + pl);
    free(emods);
    free(brot);
    free(acc);
    free(hat);
    free(erot);
    free(ext);
    return rc;
}

/* ---------------------------------------------------------------------------
 * NewMult (Sec. 5.1, Algorithm "NewMult"): Mult with its two ModDowns (the
 * key-switch's division by P and Rescale's division by q_(level-1)) merged.
 * The tensor terms b3, c3 are lifted with PModUp (times P on the q limbs, 0
 * on the P limbs) and added to the KSKInnerProd outputs before one ModDown
 * that divides by S = P q_(level-1): the special limbs are p_0..p_(K-1) and
 * q_(level-1), y_s = iNTT(x_s) [(S/s)^-1]_s, z_i = NTT(sum_s y_s [S/s]_(q_i)),
 * out_i = (x_i - z_i) [S^-1]_(q_i) for i < level - 1.  As for ModDown by P,
 * the conversion is uncorrected (no rounding offset).  Output at level - 1.
 * ------------------------------------------------------------------------- */
static void moddown_s(const oref_params *pr, const uint64_t *x, uint32_t level, uint64_t *y) {
    size_t n = (size_t)1 << pr->log_n;
    uint32_t K = pr->K, ns = K + 1, lo = level - 1;
    uint64_t *sm = (uint64_t *)malloc(sizeof(uint64_t) * ns);  /* special moduli */
    for (uint32_t k = 0; k < K; k++) sm[k] = pr->p[k];
    sm[K] = pr->q[lo];
    uint64_t *ys = (uint64_t *)malloc(sizeof(uint64_t) * n * ns);
    memcpy(ys, x + (size_t)level * n, sizeof(uint64_t) * n * K);     /* P limbs */
    memcpy(ys + (size_t)K * n, x + (size_t)lo * n, sizeof(uint64_t) * n);  /* q_(level-1) */
    for (uint32_t k = 0; k < ns; k++) {
        uint64_t m = sm[k], prod = 1;
        intt_limb(ys + (size_t)k * n, pr->log_n, m);
        for (uint32_t kk = 0; kk < ns; kk++) if (kk != k) prod = mulmod(prod, sm[kk] % m, m);
        uint64_t inv = invmod(prod, m);
        for (size_t c = 0; c < n; c++) ys[k * n + c] = mulmod(ys[k * n + c], inv, m);
    }
    uint64_t *z = (uint64_t *)malloc(sizeof(uint64_t) * n);
    for (uint32_t i = 0; i < lo; i++) {
        uint64_t qi = pr->q[i], smod = 1;
        uint64_t cst[OREF_MAX_SRC];
        for (uint32_t k = 0; k < ns; k++) {
            uint64_t prod = 1;
            for (uint32_t kk = 0; kk < ns; kk++) if (kk != k) prod = mulmod(prod, sm[kk] % qi, qi);
            cst[k] = prod;
            smod = mulmod(smod, sm[k] % qi, qi);
        }
        uint64_t sinv = invmod(smod, qi);
        for (size_t c = 0; c < n; c++) {
            u128 acc = 0;
            for (uint32_t k = 0; k < ns; k++) acc += (u128)ys[k * n + c] * cst[k];
            z[c] = (uint64_t)(acc % qi);
        }
        ntt_limb(z, pr->log_n, qi);
        for (size_t c = 0; c < n; c++) y[i * n + c] = mulmod(submod(x[i * n + c], z[c], qi), sinv, qi);
    }
    free(z);
    free(ys);
    free(sm);
}

int oref_new_mult(const oref_params *pr, const uint64_t *ct1, const uint64_t *ct2, uint32_t level,
                  const uint64_t *rlk, uint64_t *out) {
    if (check(pr, level) || level < 2) return -1;
    size_t n = (size_t)1 << pr->log_n;
    size_t pl = (size_t)level * n;
    uint32_t next = level + pr->K, beta = beta_of(pr, level);
    if (beta > pr->dnum) return -1;
    uint64_t *a3 = (uint64_t *)malloc(sizeof(uint64_t) * pl);
    uint64_t *bc = (uint64_t *)malloc(sizeof(uint64_t) * pl * 2);
    uint64_t *ext = (uint64_t *)malloc(sizeof(uint64_t) * n * next * beta);
    uint64_t *hat = (uint64_t *)malloc(sizeof(uint64_t) * n * next * 2);
    for (uint32_t i = 0; i < level; i++) {
        uint64_t q = pr->q[i];
        for (size_t c = 0; c < n; c++) {
            size_t o = i * n + c;
            uint64_t a1 = ct1[o], b1 = ct1[pl + o], a2 = ct2[o], b2 = ct2[pl + o];
            a3[o] = mulmod(a1, a2, q);
            bc[o] = addmod(mulmod(a1, b2, q), mulmod(a2, b1, q), q);
            bc[pl + o] = mulmod(b1, b2, q);
        }
    }
    int rc = oref_modup(pr, a3, level, ext);
    if (!rc) rc = oref_ksk_inner(pr, ext, level, rlk, hat);
    if (!rc) {
        /* PModUp(b3), PModUp(c3) added on the q limbs */
        for (uint32_t row = 0; row < 2; row++)
            for (uint32_t i = 0; i < level; i++) {
                uint64_t q = pr->q[i], pmod = 1;
                for (uint32_t k = 0; k < pr->K; k++) pmod = mulmod(pmod, pr->p[k] % q, q);
                uint64_t *h = hat + ((size_t)row * next + i) * n;
                for (size_t c = 0; c < n; c++) h[c] = addmod(h[c], mulmod(pmod, bc[row * pl + i * n + c], q), q);
            }
        moddown_s(pr, hat, level, out);
        moddown_s(pr, hat + (size_t)next * n, level, out + (size_t)(level - 1) * n);
    }
    free(hat);
    free(ext);
    free(bc);
    free(a3);
    return rc;
}
