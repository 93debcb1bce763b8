/* Hybrid key-switching in 32-bit words (the word-size trade-off of Sec. 5.4:
 * machine words narrower than 64 bits make every modular product cheaper,
 * at the price of more limbs for the same log2(QP)).
 *
 * The operations are those of include/hks.h (ModUp, KSKInnerProd, ModDown,
 * Rotate = Algorithm 3, HRotate = Algorithm 4), in the same layouts with
 * uint32_t words: a polynomial at level l is [l][N] limb-major canonical
 * residues in the bit-reversed evaluation order of the 64-bit library; a
 * ciphertext is [2][l][N] (a, b); a switching key [dnum][2][L+K][N].  Primes
 * satisfy 2^20 < q < 2^30 and q = 1 mod 2N, so that values up to 4q fit in
 * a word and products of two residues fit in 64 bits.  Status codes, the Galois
 * element helpers and the stream convention are those of include/hks.h.
 * The decomposition, the uncorrected fast basis conversion, the floor-style
 * ModDown and the automorphism are the same as in the 64-bit library, so
 * for the same primes both compute the same residues. */
#ifndef HKS32_H
#define HKS32_H

#include <stdint.h>

#include "hks.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hks32_ctx hks32_ctx;

typedef struct {
    uint32_t log_n;     /* 10..16 */
    uint32_t L;         /* ciphertext primes, 1..96 */
    uint32_t K;         /* special primes, alpha <= K <= 16 */
    uint32_t dnum;      /* digits; alpha = ceil(L / dnum) <= 16 */
    const uint32_t *q;  /* HOST array of L primes */
    const uint32_t *p;  /* HOST array of K primes */
} hks32_params;

/* Context: validates the primes (HKS_EINVAL otherwise), builds twiddle and
 * conversion tables on `device` and allocates the workspace of a key-switch
 * at the top level with ModDown slots for four (hoisted) rotations
 * ([L] + [dnum][L+K] + 4 ([2][L] + [2][K] + [2][L]) limbs).  Calls on one
 * context must not overlap. */
int hks32_create(const hks32_params *params, int device, hks32_ctx **out);
void hks32_destroy(hks32_ctx *ctx);

/* Forward / inverse negacyclic NTT (Sec. 2.3) of n_limbs limbs x[i]
 * modulo prime first_mod + i (q_0..q_{L-1}, p_0..p_{K-1}), in place,
 * canonical output. */
int hks32_ntt(hks32_ctx *ctx, uint32_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream);
int hks32_intt(hks32_ctx *ctx, uint32_t *x, uint32_t first_mod, uint32_t n_limbs, void *stream);

/* Rotate (Algorithm 3): (u, v) = KeySwitch(automorph(a, galois), ksk);
 * ct_out = (u, v + automorph(b, galois)).  ct [2][level][N], ksk
 * [dnum][2][L+K][N], ct_out [2][level][N], all device pointers, 16-byte
 * aligned; ct_out must not alias ct.  galois odd, below 2N. */
int hks32_rotate(hks32_ctx *ctx, const uint32_t *ct, uint32_t level, uint32_t galois, const uint32_t *ksk,
                 uint32_t *ct_out, void *stream);

/* HRotate (Algorithm 4): one ModUp of a (no automorphism; the extended
 * digits taken fully into evaluation form), then for each i < r the
 * KSKInnerProd with ksk[i] over the digits automorphed by galois[i], ModDown
 * of u and v (one sequence per four rotations), and
 * ct_out[i] = (u, v + automorph(b, galois[i])).  galois, ksk
 * and ct_out are HOST arrays of r entries (ksk[i], ct_out[i] device
 * pointers, 16-byte aligned, ct_out[i] not aliasing ct).  Same residues as
 * hks_hrotate of include/hks.h for the same primes; they differ from r calls
 * of hks32_rotate, since the automorphism follows the uncorrected basis
 * conversion.  HKS_EINVAL for r = 0 or any invalid entry (nothing runs). */
int hks32_hrotate(hks32_ctx *ctx, const uint32_t *ct, uint32_t level, uint32_t r, const uint32_t *galois,
                  const uint32_t *const *ksk, uint32_t *const *ct_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HKS32_H */
