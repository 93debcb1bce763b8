// Key-switching in 32-bit words (Sec. 5.4: the word-size trade-off).
//
// The same hybrid key-switch as the 64-bit path (ModUp, KSKInnerProd,
// ModDown, automorphism for Rotate), with residues held in 32-bit words for
// primes q < 2^30: products fit in 64 bits, so every modular product is a
// 32-bit Shoup multiply (one high and two low 32-bit multiplies) and every
// sum of products accumulates exactly in a 64-bit word.  The same log2(QP)
// needs about 5/3 as many limbs as with 50-bit primes, and each limb is half
// the bytes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace hks {
namespace w32 {

constexpr uint32_t MAXL32 = 255;  // moduli per context (uint8 indices)
constexpr uint32_t MAXS32 = 16;   // source limbs of one basis conversion
constexpr uint32_t HB32 = 4;      // rotations of one ModDown step (HRotate)

struct Shoup32 {
    uint32_t w, wp;  // wp = floor(w 2^32 / q)
};

struct Mod32 {
    uint32_t q, pad;
    uint64_t mu;  // floor(2^64 / q)
};

// Folded last inverse stage: x0' = (u + v) c, x1' = (u - v) cw.
struct Last32 {
    Shoup32 c, cw;
};

// Up to MAXL32 limbs of one launch: limb i is read at in + in_off[i] N,
// written at out + out_off[i] N, modulus mod[i], constant index cidx[i].
struct Map32 {
    uint32_t count;
    uint16_t in_off[MAXL32];
    uint16_t out_off[MAXL32];
    uint8_t mod[MAXL32];
    uint16_t cidx[MAXL32];
};

struct Ctx32 {
    int device = 0;
    uint32_t log_n = 0, n = 0, n1 = 0, n2 = 0, L = 0, K = 0, dnum = 0, alpha = 0, M = 0;
    std::vector<uint32_t> mods;          // q_0..q_{L-1}, p_0..p_{K-1}
    Shoup32 *tw_fwd = nullptr, *tw_inv = nullptr;  // [M][N], psi^(+-brv(i))
    Mod32 *mc = nullptr;                 // [M]
    Last32 *li_plain = nullptr;          // [M]: N^-1
    Last32 *li_modup = nullptr;          // [L+1][L]: N^-1 (Qt_j / q_i)^-1 at level l
    Last32 *li_moddown = nullptr;        // [K]: N^-1 (P / p_k)^-1
    uint32_t *conv_modup = nullptr;      // per level: [beta][E][alpha] of [Qt_j / q_i]_t
    std::vector<size_t> conv_modup_off;  // [L+1]
    uint32_t *conv_moddown = nullptr;    // [L][K] of [P / p_k]_{q_i}
    Shoup32 *pinv = nullptr;             // [L]: P^-1 mod q_i
    // workspace, allocated at create: sized for the top level and HB32
    // rotations per ModDown step; the per-rotation slots of ws_uv are
    // [2][level][N] at stride 2 level N, those of ws_p [2][K][N]
    uint32_t *ws = nullptr;
    uint32_t *ws_y = nullptr;    // [L][N]             coefficient-form input limbs
    uint32_t *ws_ext = nullptr;  // [dnum][L+K][N]     extended digits
    uint32_t *ws_uv = nullptr;   // [HB32][2][L][N]    KSKInnerProd on the q limbs
    uint32_t *ws_p = nullptr;    // [HB32][2][K][N]    P limbs of u, v
    uint32_t *ws_z = nullptr;    // [HB32][2][L][N]    ModDown corrections
};

// Launchers (ks32.hip).  The limbs of a launch follow its map, repeated for
// `ys` polynomials at strides in_ys / out_ys words; the inverse column pass
// takes `fold`.
hipError_t launch32_fwd_cols(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, hipStream_t s,
                             uint32_t ys = 1, size_t in_ys = 0, size_t out_ys = 0);
hipError_t launch32_fwd_rows(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, hipStream_t s);
hipError_t launch32_inv_rows(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, uint32_t galois,
                             hipStream_t s);
hipError_t launch32_inv_cols(const Ctx32 &c, const Map32 &m, const uint32_t *in, uint32_t *out, const Last32 *fold,
                             hipStream_t s, uint32_t ys = 1, size_t in_ys = 0, size_t out_ys = 0);
// ModUp's NewLimb at `level`: ext[j][t] for t outside digit j, from y.
hipError_t launch32_conv_modup(const Ctx32 &c, const uint32_t *y, uint32_t level, uint32_t *ext, hipStream_t s);
// ModDown's NewLimb: z[p][i] (i < level, z at stride L N) from the K P limbs
// pc[p][k], p < polys.
hipError_t launch32_conv_moddown(const Ctx32 &c, const uint32_t *pc, uint32_t level, uint32_t polys, uint32_t *z,
                                 hipStream_t s);
// Forward row pass of ext's new limbs + KSKInnerProd (own limbs gathered from
// `a` through galois) + inverse row pass of the P limbs: uq [2][level][N],
// pc [2][K][N].  With `direct`, ext's new limbs are in evaluation form
// already and are gathered through galois as well (no row pass).
hipError_t launch32_ksk(const Ctx32 &c, const uint32_t *ext, bool direct, const uint32_t *a, uint32_t galois,
                        uint32_t level, const uint32_t *ksk, uint32_t *uq, uint32_t *pc, hipStream_t s);
// ModDown's last step on the forward row pass of z, for nrot <= HB32
// ciphertexts r: polynomial p of r is y = 2 r + p, z at z + y L N, u at
// uq + y level N; outs[r][p] = (u - z) P^-1, plus b gathered through
// gals[r] for p = 1.
hipError_t launch32_rows_epi(const Ctx32 &c, uint32_t level, const uint32_t *z, const uint32_t *uq,
                             const uint32_t *b, uint32_t nrot, uint32_t *const *outs, const uint32_t *gals,
                             hipStream_t s);

int build_tables32(Ctx32 &c);
void free_tables32(Ctx32 &c);

}  // namespace w32
}  // namespace hks
