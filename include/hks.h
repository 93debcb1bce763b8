/*
 * hks.h -- C ABI of the MI355X (gfx950) CKKS hybrid key-switching library.
 *
 * Operations follow de Castro et al., "Does Fully Homomorphic Encryption
 * Need Compute Acceleration?" (arXiv 2112.06396):
 *   - ModUp, ModDown, Decomp, KSKInnerProd, Automorph: Table "CKKS
 *     Subroutines" (Sec. 2.4) and the switching-key shape, Eq. (kskShape);
 *   - ModUp as iNTT -> NewLimb (basis conversion) -> NTT: Algorithm "ModUp";
 *   - Rotate: Algorithm 3; HRotate (hoisted rotations): Algorithm 4;
 *   - PtMult with Rescale: Algorithm 1; Mult with relinearization: Algorithm 2;
 *   - NTT / evaluation representation: Sec. 2.3; RNS limbs: Sec. 2.2.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Moduli.   A context holds L ciphertext primes q_0..q_{L-1} and K special
 *            primes p_0..p_{K-1} (P = prod p_k).  Every prime must satisfy
 *            2^49 < q < 2^50 and q = 1 mod 2N, and all must be distinct.
 *            A "modulus index" numbers them 0..L-1 (q_i) then L..L+K-1 (p_k).
 *  Digits.   alpha = ceil(L / dnum) limbs per digit; at level l (l limbs
 *            q_0..q_{l-1} present) beta = ceil(l / alpha) digits, digit j
 *            holding limbs [j*alpha, min((j+1)*alpha, l)).  K >= alpha.
 *  Layout.   Polynomials are limb-major: [limbs][N] uint64, one limb per
 *            modulus, residues canonical in [0, q).  Ciphertexts are (a, b)
 *            as [2][l][N]; decryption is a*s + b.  The evaluation form holds
 *            slot j = a(psi^(2 brv(j) + 1)) (bit-reversed order), psi =
 *            nu^((q-1)/2N) with nu the least quadratic non-residue mod q.
 *            Extended polynomials (over Q_l U P) order their limbs
 *            q_0..q_{l-1}, p_0..p_{K-1}.
 *  Keys.     Switching keys are [dnum][2][L+K][N] (row 0 = a_j, row 1 =
 *            b_j), the limb of q_i at index i and of p_k at index L+k; at
 *            level l only limbs [0,l) U [L,L+K) of digits j < beta are read.
 *  Memory.   All uint64_t* data arguments are DEVICE pointers on the
 *            context's device, owned by the caller, 16-byte aligned.  The
 *            library never frees or retains them.  Outputs must not alias
 *            inputs unless a call says "in place".
 *  Streams.  `stream` is a hipStream_t (NULL = default stream).  Calls only
 *            enqueue work and return; the caller synchronizes.  A context
 *            owns one workspace: calls on one context must not run
 *            concurrently on different streams.
 *  Errors.   Every int-returning call returns HKS_OK (0) or a negative
 *            status; no exception crosses the ABI and nothing aborts.  On an
 *            error no work has been enqueued, except HKS_EHIP, which reports
 *            a failed HIP launch.  hks_strerror() names a status.
 */
#ifndef HKS_H
#define HKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HKS_OK 0
#define HKS_EINVAL (-1)       /* bad argument: level, galois, pointer, size, parameters */
#define HKS_ENOMEM (-2)       /* device or host allocation failed */
#define HKS_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define HKS_EUNSUPPORTED (-4) /* valid request outside what the library supports */
#define HKS_ERANGE (-5)       /* an input residue is not below its modulus (checks on) */
#define HKS_ESCRATCH (-6)     /* the call needs more than the allocation-free scratch */

/* hks_query keys */
#define HKS_Q_N 1              /* ring degree N */
#define HKS_Q_ALPHA 2          /* limbs per digit */
#define HKS_Q_BETA 3           /* digits at `level` */
#define HKS_Q_KSK_WORDS 4      /* uint64 words of one switching key, dnum*2*(L+K)*N */
#define HKS_Q_WORKSPACE_BYTES 5/* device workspace owned by the context */
#define HKS_Q_MODULUS 6        /* modulus with index `level` (0..L+K-1) */
#define HKS_Q_L 7
#define HKS_Q_K 8
#define HKS_Q_DNUM 9
#define HKS_Q_BATCH_CAP 10     /* ciphertexts (or rotations) per batched launch step */
#define HKS_Q_NOALLOC_BYTES 11 /* scratch bytes hks_rotate_noalloc uses at `level` */
#define HKS_Q_NOALLOC_MAX_BYTES 12 /* size of the allocation-free scratch */

/* Size of the device array that serves as hks_rotate_noalloc's workspace
 * (one per GPU, held from the library's first use on that GPU until the
 * process ends). */
#define HKS_NOALLOC_SCRATCH_BYTES (128ull << 20)

typedef struct hks_ctx hks_ctx;

typedef struct {
    uint32_t log_n;       /* 10..16 */
    uint32_t L;           /* ciphertext primes, 1..48 */
    uint32_t K;           /* special primes, alpha..16 */
    uint32_t dnum;        /* digits of the switching key, 1..L */
    const uint64_t *q;    /* host array [L] */
    const uint64_t *p;    /* host array [K] */
    uint32_t max_batch;   /* ciphertexts (or rotations) per batched launch step,
                             0..16 (0 = 1).  The workspace holds one slot per
                             step entry: (6L + dnum(L+K) + 2(L+K) + 2K + 2L) N
                             words each, plus 2 L N + 2 N words shared. */
} hks_params;

/* ---------------------------------------------------------------- host helpers */

/* Primes of the form 2^bits - k*2^log_step + 1 (k = 1, 2, ...), descending,
 * primality by deterministic Miller-Rabin.  bits = 50, log_step = log_n + 1
 * (or larger) give primes valid for this library.  `out` is a host array of
 * `count` words.  Returns HKS_OK or HKS_EINVAL. */
int hks_gen_primes(uint32_t bits, uint32_t log_step, uint32_t count, uint64_t *out);

/* Galois element g with Rotate(ct, g) realizing the paper's rotation phi_k
 * (Sec. 2.1: phi_1 moves slot j-1 to slot j) under slots m(zeta^(5^j)):
 * g = 5^(-k) mod 2N.  Negative k rotates the other way. */
uint32_t hks_galois_for_rotation(int32_t k, uint32_t log_n);

/* Galois element of complex conjugation, 2N - 1 (Conjugate, Table
 * "CKKS FHE API": same implementation as Rotate). */
uint32_t hks_galois_conjugate(uint32_t log_n);

const char *hks_strerror(int status);

/* ---------------------------------------------------------------- context */

/* Validates the parameters, builds twiddle and conversion tables on `device`
 * (HIP ordinal) and allocates the workspace.  *out is set only on HKS_OK. */
int hks_create(const hks_params *params, int device, hks_ctx **out);

/* Frees tables and workspace (synchronizes the device first).  NULL is a no-op. */
void hks_destroy(hks_ctx *ctx);

/* Reads one HKS_Q_* value into *out. */
int hks_query(const hks_ctx *ctx, int key, uint32_t level, uint64_t *out);

/* ---------------------------------------------------------------- polynomial calls */

/* In place forward NTT (Sec. 2.3) of n_limbs consecutive limbs of x, limb i
 * reduced by the modulus with index first_mod + i (coefficient -> evaluation). */
int hks_ntt(hks_ctx *ctx, uint64_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream);

/* In place inverse NTT (evaluation -> coefficient), same arguments. */
int hks_intt(hks_ctx *ctx, uint64_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream);

/* Automorph X -> X^galois (Table "CKKS Subroutines"), galois odd in [1, 2N).
 * eval_domain != 0: slot permutation of evaluation-form limbs; else the
 * coefficient map with negation.  y = psi_g(x), n_limbs limbs with moduli
 * first_mod..first_mod+n_limbs-1; x and y must not overlap. */
int hks_automorph(hks_ctx *ctx, const uint64_t *x, uint64_t *y, uint32_t first_mod,
                  uint32_t n_limbs, uint32_t galois, int eval_domain, void *stream);

/* ModUp of every digit of a (Decomp_beta then ModUp, Table "CKKS Subroutines",
 * Algorithm "ModUp"): a [level][N] evaluation form -> ext [beta][level+K][N]
 * evaluation form.  Fast basis conversion without correction: digit j's own
 * limbs are copied, the others hold sum_i [x_i (Qt_j/q_i)^-1]_{q_i} (Qt_j/q_i). */
int hks_modup(hks_ctx *ctx, const uint64_t *a, uint32_t level, uint64_t *ext, void *stream);

/* KSKInnerProd (Table "CKKS Subroutines"): uv[0] = sum_j ext[j]*ksk[j][0],
 * uv[1] = sum_j ext[j]*ksk[j][1], limb-wise.  ext [beta][level+K][N],
 * ksk [dnum][2][L+K][N], uv [2][level+K][N]. */
int hks_ksk_inner(hks_ctx *ctx, const uint64_t *ext, uint32_t level, const uint64_t *ksk,
                  uint64_t *uv, void *stream);

/* ModDown_{B,K} (Table "CKKS Subroutines"): x [level+K][N] -> y [level][N],
 * y = (x - sum_k [iNTT(x_{p_k}) (P/p_k)^-1]_{p_k} (P/p_k)) * P^-1 (no rounding offset). */
int hks_moddown(hks_ctx *ctx, const uint64_t *x, uint32_t level, uint64_t *y, void *stream);

/* KeySwitch: Decomp -> ModUp -> KSKInnerProd -> ModDown (u), ModDown (v).
 * d [level][N] -> uv [2][level][N]. */
int hks_keyswitch(hks_ctx *ctx, const uint64_t *d, uint32_t level, const uint64_t *ksk,
                  uint64_t *uv, void *stream);

/* Rotate (Algorithm 3): (a_r, b_r) = Automorph(ct, galois); (u, v) =
 * KeySwitch(a_r, ksk); ct_out = (u, v + b_r).  ct, ct_out [2][level][N]. */
int hks_rotate(hks_ctx *ctx, const uint64_t *ct, uint32_t level, uint32_t galois,
               const uint64_t *ksk, uint64_t *ct_out, void *stream);

/* hks_rotate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and bits as hks_rotate, but the call's workspace is
 * the library's allocation-free scratch, a fixed device array of
 * HKS_NOALLOC_SCRATCH_BYTES per GPU (128 MiB), instead of the context's
 * workspace.  The call allocates nothing (no hipMalloc, hipFree or heap use;
 * with the profiling hooks of hks_prof_enable off).
 * A Rotate at `level` needs N (5 level + 2 K + beta (L + K)) words
 * (hks_query HKS_Q_NOALLOC_BYTES): at N = 2^16, L = 24, K = 8, dnum = 3 every
 * level fits; a larger request returns HKS_ESCRATCH with nothing enqueued.
 * Every call on one GPU shares that GPU's scratch, whatever its context:
 * calls that overlap in time on one GPU (other streams, other host threads,
 * other contexts) race and give wrong results; calls on one stream are
 * ordered and safe.  Nothing needs to start at zero: each call writes every
 * scratch word it reads.  HKS_EUNSUPPORTED for a device index >= 64. */
int hks_rotate_noalloc(hks_ctx *ctx, const uint64_t *ct, uint32_t level, uint32_t galois,
                       const uint64_t *ksk, uint64_t *ct_out, void *stream);

/* HRotate (Algorithm 4): ModUp of a once, then for each i < r: automorph the
 * extended digits by galois[i], KSKInnerProd with ksk[i], ModDown x2, add the
 * automorphed b.  galois, ksk, ct_out are HOST arrays of r entries (ksk[i] and
 * ct_out[i] device pointers).  Bits differ from r calls of hks_rotate (the
 * automorphism is applied after the uncorrected conversion).  Rotations are
 * processed max_batch at a time, each step in one KSKInnerProd launch and
 * one ModDown sequence. */
int hks_hrotate(hks_ctx *ctx, const uint64_t *ct, uint32_t level, uint32_t r,
                const uint32_t *galois, const uint64_t *const *ksk, uint64_t *const *ct_out,
                void *stream);

/* PtMatVecMult with the ModDown hoisted (Sec. 5.2, Algorithm
 * "PtMatVecMult"): ct_out = sum_i M_i * Rotate_{galois[i]}(ct) computed as one
 * ModUp of a, per i the automorphed extended digits through KSKInnerProd
 * with ksk[i], multiplied by M_i together with P * b_rot over Q_level U P and
 * summed, then a single ModDown.  pt[i] is M_i over the extended basis,
 * [level + K][N] evaluation form (residues mod q_0..q_{level-1},
 * p_0..p_{K-1}; not multiplied by P).  galois, ksk, pt are HOST arrays of
 * r <= 64 entries (device pointers).  ksk[i] = NULL with galois[i] = 1 is
 * the diagonal without rotation (offset 0 of a factored DFT matrix, Sec. 3):
 * its term is M_i * (P a, P b), no key switch.  The result carries the
 * product's scale (no Rescale). */
int hks_ptmatvec(hks_ctx *ctx, const uint64_t *ct, uint32_t level, uint32_t r, const uint32_t *galois,
                 const uint64_t *const *ksk, const uint64_t *const *pt, uint64_t *ct_out, void *stream);

/* Rotate of n_ct independent ciphertexts at one level (same semantics and
 * bits as n_ct calls of hks_rotate; batching as in Sec. 2.4 and 5.2).  ct,
 * galois, ksk, ct_out are HOST arrays of n_ct entries; galois elements and
 * keys may differ per ciphertext.  Up to max_batch ciphertexts share every
 * launch of a step; the blocks of one key tile run on one XCD, so a key
 * shared by the step is streamed from HBM once.  HKS_EINVAL if an output
 * equals any input or another output. */
int hks_batch_rotate(hks_ctx *ctx, uint32_t n_ct, const uint64_t *const *ct, uint32_t level,
                     const uint32_t *galois, const uint64_t *const *ksk, uint64_t *const *ct_out,
                     void *stream);

/* Rotate of n_ct ciphertexts at levels of uneven limb count, levels[i] for
 * ciphertext i (1..L), in shared launches: one launch sequence serves up to
 * max_batch ciphertexts whatever their levels (the batching of a
 * bootstrapping trace's descending levels, Sec. 3, and of a serving mix).
 * Same bits as hks_rotate on each ciphertext at its level.  ct[i] is
 * [2][levels[i]][N], ct_out[i] likewise.  seeds NULL: ksk[i] are full keys;
 * else ksk[i] holds the rows b_j of the seeded key seeds[i] (as in
 * hks_rotate_seeded).  ct, levels, galois, seeds, ksk, ct_out are HOST
 * arrays of n_ct entries.  HKS_EINVAL if an output equals any input or
 * another output, or a level is outside [1, L]. */
int hks_batch_rotate_mixed(hks_ctx *ctx, uint32_t n_ct, const uint64_t *const *ct, const uint32_t *levels,
                           const uint32_t *galois, const uint64_t *seeds, const uint64_t *const *ksk,
                           uint64_t *const *ct_out, void *stream);

/* Mult + relinearization (Algorithm 2) of n pairs at levels of uneven limb
 * count, pair i at levels[i], in shared launches; same bits as
 * hks_mult_relin per pair.  ct1[i], ct2[i] are [2][levels[i]][N]; ct_out[i]
 * is [2][levels[i] - 1][N] with rescale (levels[i] >= 2), else
 * [2][levels[i]][N].  seeds as in hks_batch_rotate_mixed. */
int hks_batch_mult_relin_mixed(hks_ctx *ctx, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                               const uint32_t *levels, const uint64_t *seeds, const uint64_t *const *rlk,
                               int rescale, uint64_t *const *ct_out, void *stream);

/* ---------------------------------------------------------------- seeded keys/* ---------------------------------------------------------------- seeded keys
 * Key compression (Sec. 5.3): a seeded switching key stores only its rows b_j,
 * ksk_b [dnum][L+K][N]; the uniform rows a_j are regenerated on the device
 * from a 64-bit seed.  Entry (j, kappa, i) of a_j, for key limb kappa and
 * slot i, is the low 96 bits c0 + c1 2^32 + c2 2^64 of Philox4x32-10 (Salmon
 * et al., SC 2011) at counter (i, kappa, j, 0x4B53) and key (seed mod 2^32,
 * seed >> 32), reduced mod the limb's prime.  Halves the key bytes a
 * key-switch streams. */

/* The rows a_j of the seeded key `seed`: a [dnum][L+K][N] (device). */
int hks_expand_key_a(hks_ctx *ctx, uint64_t seed, uint64_t *a, void *stream);

/* hks_rotate with the seeded key (seed, ksk_b); same bits as hks_rotate with
 * the full key whose rows are (hks_expand_key_a(seed), ksk_b). */
int hks_rotate_seeded(hks_ctx *ctx, const uint64_t *ct, uint32_t level, uint32_t galois, uint64_t seed,
                      const uint64_t *ksk_b, uint64_t *ct_out, void *stream);

/* hks_batch_rotate with seeded keys: seeds and ksk_b are HOST arrays of n_ct
 * entries (ksk_b[i] a device pointer). */
int hks_batch_rotate_seeded(hks_ctx *ctx, uint32_t n_ct, const uint64_t *const *ct, uint32_t level,
                            const uint32_t *galois, const uint64_t *seeds, const uint64_t *const *ksk_b,
                            uint64_t *const *ct_out, void *stream);

/* hks_batch_mult_relin with seeded relinearization keys: seeds and rlk_b are
 * HOST arrays of n entries, rlk_b[i] the rows b_j [dnum][L+K][N] of seeded
 * key seeds[i] (device).  Same bits as hks_batch_mult_relin with the full
 * keys (hks_expand_key_a(seeds[i]), rlk_b[i]). */
int hks_batch_mult_relin_seeded(hks_ctx *ctx, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                                uint32_t level, const uint64_t *seeds, const uint64_t *const *rlk_b, int rescale,
                                uint64_t *const *ct_out, void *stream);

/* Rescale = ModDown_{B,1} (Sec. 2.4, rounding to nearest): divide by
 * q_{level-1}.  ct [2][level][N] -> ct_out [2][level-1][N], level >= 2. */
int hks_rescale(hks_ctx *ctx, const uint64_t *ct, uint32_t level, uint64_t *ct_out, void *stream);

/* PtMult (Algorithm 1): (a*pt, b*pt) limb-wise, pt [level][N] evaluation
 * form, then Rescale if rescale != 0.  ct_out [2][level or level-1][N]. */
int hks_ptmult(hks_ctx *ctx, const uint64_t *ct, const uint64_t *pt, uint32_t level, int rescale,
               uint64_t *ct_out, void *stream);

/* Mult (Algorithm 2): (a3, b3, c3) = (a1 a2, a1 b2 + a2 b1, b1 b2); (u, v) =
 * KeySwitch(a3, rlk); (b3 + u, c3 + v); then Rescale if rescale != 0. */
int hks_mult_relin(hks_ctx *ctx, const uint64_t *ct1, const uint64_t *ct2, uint32_t level,
                   const uint64_t *rlk, int rescale, uint64_t *ct_out, void *stream);

/* Mult (Algorithm 2) of n independent pairs at one level (same semantics and
 * bits as n calls of hks_mult_relin).  ct1, ct2, rlk, ct_out are HOST arrays
 * of n device pointers; up to max_batch pairs share the key-switch launches
 * of a step.  HKS_EINVAL if an output equals any input or another output. */
int hks_batch_mult_relin(hks_ctx *ctx, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                         uint32_t level, const uint64_t *const *rlk, int rescale, uint64_t *const *ct_out,
                         void *stream);

/* NewMult (Sec. 5.1): Mult with rescale = 1 where the key-switch ModDown
 * and the Rescale are one ModDown by S = P q_{level-1}.  The KSKInnerProd
 * kernel adds P b3 and P c3 to (u, v) on the q limbs (b3, c3 as in
 * hks_mult_relin), the q_{level-1} limb joins the K special limbs, and the
 * ModDown basis-converts those K+1 limbs, so the output ct_out
 * [2][level-1][N] is floor((P (b3, c3) + (u, v)) / S) with the uncorrected
 * conversion's small error.  Its bits differ from hks_mult_relin(..., 1, ...)
 * by a few units (the two roundings become one); the difference decrypts
 * within the scheme's error.  level >= 2; ct_out must not alias ct1 or ct2.
 * HKS_EUNSUPPORTED when K + 1 > 16. */
int hks_new_mult(hks_ctx *ctx, const uint64_t *ct1, const uint64_t *ct2, uint32_t level, const uint64_t *rlk,
                 uint64_t *ct_out, void *stream);

/* NewMult of n pairs at one level in shared launches (up to max_batch pairs
 * per step); same bits as hks_new_mult per pair.  ct1, ct2, rlk, ct_out are
 * HOST arrays of n entries (device pointers); ct_out[i] is
 * [2][level - 1][N].  HKS_EINVAL if an output equals any input or another
 * output. */
int hks_batch_new_mult(hks_ctx *ctx, uint32_t n, const uint64_t *const *ct1, const uint64_t *const *ct2,
                       uint32_t level, const uint64_t *const *rlk, uint64_t *const *ct_out, void *stream);

/* Encode (the CKKS canonical embedding, Sec. 2.1; the plaintexts of the
 * factored DFT's diagonals in bootstrapping, Sec. 3).  slots: DEVICE array of
 * N/2 complex values as interleaved fp64 (re, im), 16-byte aligned; slot j is
 * the plaintext's value at zeta^(5^j mod 2N), zeta = exp(i pi / N).  With
 * w = V^H z / (N/2) (V[j, k] = zeta^(5^j k)), the plaintext's coefficients
 * are m_k = round(scale Re w_k), m_(k+N/2) = round(scale Im w_k) (round half
 * to even, fp64), reduced mod q_0..q_{level-1} and, if with_p != 0, also
 * p_0..p_{K-1}; pt_out [level (+K)][N] evaluation form.  Requires
 * scale * |w_k| < 2^62 (larger values give undefined residues).  The
 * transform runs in fp64 butterflies on the device; its rounding can differ
 * from another fp64 evaluation order by one unit where scale * w_k lies
 * within the rounding error of a half-integer.  Uses the context's
 * workspace (stream-ordered like every call). */
int hks_encode(hks_ctx *ctx, const double *slots, double scale, uint32_t level, int with_p, uint64_t *pt_out,
               void *stream);

/* Add (Table "CKKS FHE API"): out = x + y limb-wise for n_poly (1..3)
 * polynomials of level limbs each, [n_poly][level][N]; out may be x or y
 * (elementwise, in place allowed). */
int hks_add(hks_ctx *ctx, const uint64_t *x, const uint64_t *y, uint32_t level, uint32_t n_poly,
            uint64_t *out, void *stream);

/* ---------------------------------------------------------------- input checks */

/* Canonical-range checks.  With on != 0 every call that reads residues
 * first checks on the device that each input word (ciphertexts,
 * plaintexts, keys, NTT operands, over the limbs the call reads) is below
 * its modulus, and returns HKS_ERANGE without enqueuing its work when one is
 * not.  The check copies its verdict to the host and synchronizes the
 * stream, so it is a debugging aid: a call with checks on returns
 * HKS_EUNSUPPORTED on a capturing stream.  Off by default; the environment
 * variable HKS_DEBUG_CHECK_CANONICAL (non-empty, not "0") turns it on for
 * contexts created afterwards. */
int hks_set_check(hks_ctx *ctx, int on);

/* ---------------------------------------------------------------- launch plans */

/* Launch-shape choices of a context: how a launch's work is laid over the
 * chip (elements per thread, grouping of conversion targets, block order
 * across the 8 XCDs).  No field changes a result: every plan computes the
 * same residues.  hks_create sets the defaults given below; the tuner
 * (paper_2112_06396_amd/tune.py) times candidate plans on a workload and
 * keeps the fastest per device and shape. */
typedef struct {
    /* NTT passes, indexed by class HKS_K_NTT_FWD_COLS .. HKS_K_NTT_INV_COLS:
     * a launch runs 16 elements per thread when it holds at least this many
     * waves of 16-element threads, else 8 (one more LDS exchange, twice the
     * waves).  0 = always 16, 0xFFFFFFFF = always 8.  Defaults 6144, except
     * 0xFFFFFFFF for the forward row pass. */
    uint32_t e16_min_waves[4];
    /* NewLimb (ModUp and ModDown conversions): a launch of at most
     * conv_group_max_batch ciphertexts splits its target limbs into groups of
     * about conv_group_limbs (one block row per group); wider launches keep
     * all targets in one group.  Defaults 8 and 2; conv_group_limbs 1..64,
     * conv_group_max_batch any value (0: never split). */
    uint32_t conv_group_limbs;
    uint32_t conv_group_max_batch;
    /* Batched launches: 1 deals the entries of one (limb, row tile) to one
     * XCD one after another, so that what they share (row-pass twiddles,
     * a key tile shared by a batch) is fetched into that XCD's L2 once;
     * 0 orders blocks entry by entry.  Defaults 1 and 1. */
    uint32_t row_xcd_order;  /* batched NTT row passes */
    uint32_t ksk_xcd_order;  /* batched KSKInnerProd */
    /* Tile shapes of the two-pass NTT (Sec. 2.3): N = 2^n1 x 2^n2 with the
     * column pass over stages 0..n1-1 and the row pass over the rest.  n1:
     * 0 = log2(N)/2 (the default), else any value with 5 <= n1 <= 9 and
     * 5 <= log2(N) - n1 <= 9.  col_lines: columns per column-pass block (8,
     * 16 or 32; default 16); row_lines: rows per row-pass block (4, 8 or 16;
     * default 8); both apply to passes of 7 or more stages whose block stays
     * within 1024 threads, the defaults elsewhere.  The key-switch kernel
     * keeps 8 rows per block. */
    uint32_t n1;
    uint32_t col_lines;
    uint32_t row_lines;
} hks_plan;

/* Copies the context's plan into *out. */
int hks_get_plan(hks_ctx *ctx, hks_plan *out);
/* Replaces the plan for the calls that follow (enqueued work keeps the plan
 * it was launched with).  HKS_EINVAL, plan unchanged, if conv_group_limbs is
 * 0 or above 64, an order flag is above 1, n1 is outside its range, or a
 * width is not one of its three values. */
int hks_set_plan(hks_ctx *ctx, const hks_plan *plan);

/* ---------------------------------------------------------------- graphs */

/* Call sequences recorded once and replayed as one HIP graph (a
 * bootstrapping-shaped trace of many key-switches, Sec. 3).  The library's
 * calls allocate nothing and set no memory, so every node of such a graph
 * is a kernel launch (or the encoder's device copy).  hks_graph_begin
 * starts capturing `stream` (a created stream, not the legacy default one;
 * capture mode: this thread only); the calls that follow on that stream are
 * recorded, not run; hks_graph_end stops the capture and instantiates the
 * graph; hks_graph_launch replays it on `stream`.  The recorded calls read
 * and write the same device buffers at every replay. */
typedef struct hks_graph hks_graph;
int hks_graph_begin(void *stream);
int hks_graph_end(void *stream, hks_graph **out);
int hks_graph_launch(hks_graph *graph, void *stream);
void hks_graph_destroy(hks_graph *graph);

/* ---------------------------------------------------------------- kernel timing */

/* Kernel classes for hks_prof_* (bit i of a mask selects class i). */
#define HKS_K_NTT_FWD_COLS 0 /* forward NTT, column pass (stages 0..n1-1) */
#define HKS_K_NTT_FWD_ROWS 1 /* forward NTT, row pass (stages n1..n-1) */
#define HKS_K_NTT_INV_ROWS 2 /* inverse NTT, row pass (+ automorph gather) */
#define HKS_K_NTT_INV_COLS 3 /* inverse NTT, column pass (+ folded scale) */
#define HKS_K_CONV 4         /* basis conversion (NewLimb) */
#define HKS_K_KSK 5          /* KSKInnerProd */
#define HKS_K_MODDOWN_EPI 6  /* ModDown final step */
#define HKS_K_AUTOMORPH 7    /* standalone automorph / limb copy */
#define HKS_K_ELEMENTWISE 8  /* PtMult, tensor, Rescale steps */
#define HKS_K_COUNT 9

/* Measurement aid.  While bit k of `mask` is set, every launch of kernel
 * class k records a hipEvent pair on the launch stream; hks_prof_read()
 * waits for the recorded events and returns the summed milliseconds and the
 * launch count of class k since the last hks_prof_enable() call.  mask = 0
 * turns recording off.  The events are timing-only (hipEventDisableSystemFence:
 * no system-scope cache writeback at the record), created on the host side
 * only; no device memory is allocated. */
int hks_prof_enable(hks_ctx *ctx, uint32_t mask);
int hks_prof_read(hks_ctx *ctx, int kernel_class, double *ms, uint64_t *launches);

/* Measurement aid: the device's rate of modular products, as *per_s
 * products per second.  One kernel at full occupancy runs 8 independent
 * chains of the lazy Shoup product (x w mod q in [0, 2q) with a precomputed
 * quotient: the NTT butterfly's multiply, Sec. 2.2) for `iters` rounds per
 * thread, timed with HIP events on `stream`; the call waits for it.  It
 * writes one word per thread into the context's workspace, so it must not
 * overlap other calls on the context. */
int hks_modmul_rate(hks_ctx *ctx, uint32_t iters, void *stream, double *per_s);

#ifdef __cplusplus
}
#endif

#endif /* HKS_H */
