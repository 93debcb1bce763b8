// Internal structures of the HIP key-switching library: the context, its
// device tables, and the kernel-launch entry points shared by the host files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/hks.h"

namespace hks {

constexpr int MAXL = 128;  // limbs per launch descriptor
constexpr int MAXB = 32;   // batch entries (polynomials) per launch
constexpr int MAXCT = 16;  // ciphertexts per batched key-switch step (two polynomials each)
constexpr int MAXROT = 64; // rotations of one PtMatVecMult launch

// A list of limbs for one launch.  Limb i is read at in_base + in_off[i]*N
// (+ blockIdx.y * in_bstride for batches), written at out_base + out_off[i]*N,
// reduced by modulus mod[i], and uses constant-table entry cidx[i]; dig[i] is
// the digit a limb of extended digits belongs to (NO_DIGIT otherwise).
constexpr uint8_t NO_DIGIT = 0xFF;
struct LimbMap {
    uint32_t count;
    uint16_t in_off[MAXL];
    uint16_t out_off[MAXL];
    uint8_t mod[MAXL];
    uint16_t cidx[MAXL];
    uint8_t dig[MAXL];
};

// Per batch entry b of a pass launch: where its limbs are read and written.
// Limb i of entry b is read at in[b] + in_off[i]*N and written at
// out[b] + out_off[i]*N.  IO_GATHER reads through the automorph galois[b];
// the ModDown epilogue reads u at uq[b] + cidx[i]*N and adds add[b] +
// cidx[i]*N gathered through add_galois[b] (add[b] null: nothing added).
// Entries of one launch may sit at different levels: entry b skips the limbs
// of q primes at or above lvl[b] and the limbs of digits at or above nbeta[b]
// (0: no limit), and reads the folded constants at cidx[i] + cbase[b].
struct BatchIo {
    const uint64_t *in[MAXB];
    uint64_t *out[MAXB];
    const uint64_t *uq[MAXB];
    const uint64_t *add[MAXB];
    uint32_t galois[MAXB];
    uint32_t add_galois[MAXB];
    uint8_t lvl[MAXB];
    uint8_t nbeta[MAXB];
    uint16_t cbase[MAXB];
};

// Entries at fixed strides from two bases (workspace buffers).
inline BatchIo strided_io(const uint64_t *in, size_t in_bstride, uint64_t *out, size_t out_bstride,
                          uint32_t batch) {
    BatchIo io{};
    for (uint32_t b = 0; b < batch && b < (uint32_t)MAXB; ++b) {
        io.in[b] = in + b * in_bstride;
        io.out[b] = out + b * out_bstride;
        io.galois[b] = 1;
        io.add_galois[b] = 1;
    }
    return io;
}

// Per-modulus constants.
struct ModC {
    uint64_t q;
    uint64_t mu;  // floor(2^112 / q), Barrett for 128-bit values
    uint64_t nq;  // 2^64 - q (held in the table so that products add instead of subtract)
    uint64_t qi;  // -q^-1 mod 2^64 (Montgomery reduction)
};

// Constant pair for Shoup multiplication: (w, floor(w * 2^64 / q)).
struct Shoup {
    uint64_t w, wp;
};

struct Cplx {
    double re, im;
};

// Folded last inverse-NTT stage: multiply the sum by c and the difference by
// c * W^-1 (W the stage-0 twiddle), c = N^-1 * scale.
struct LastInv {
    Shoup c, cw;
};

// The launch plan hks_create starts from (include/hks.h, hks_plan).
inline hks_plan default_plan() {
    hks_plan p{};
    for (int i = 0; i < 4; ++i) p.e16_min_waves[i] = 6 * 1024;
    // the forward row pass (ModDown's last pass with its epilogue) measured
    // faster with 8 elements per thread at every batch size
    p.e16_min_waves[HKS_K_NTT_FWD_ROWS] = 0xFFFFFFFFu;
    p.conv_group_limbs = 8;
    p.conv_group_max_batch = 2;
    p.row_xcd_order = 1;
    p.ksk_xcd_order = 1;
    p.n1 = 0;
    p.col_lines = 16;
    p.row_lines = 8;
    return p;
}

// The NTT split a plan asks for at ring degree 2^log_n (0 if out of range).
inline uint32_t plan_n1(const hks_plan &p, uint32_t log_n) {
    const uint32_t n1 = p.n1 ? p.n1 : log_n / 2;
    return (n1 >= 5 && n1 <= 9 && log_n >= n1 + 5 && log_n <= n1 + 9) ? n1 : 0;
}

struct Ctx {
    int device = 0;
    hks_plan plan = default_plan();
    uint32_t log_n = 0, n = 0, L = 0, K = 0, dnum = 0, alpha = 0, M = 0;
    uint32_t n1 = 0, n2 = 0;  // NTT split: N = 2^n1 * 2^n2 (columns of 2^n1, rows of 2^n2)
    std::vector<uint64_t> mods;  // [M]: q_0..q_{L-1}, p_0..p_{K-1}

    // device tables
    Shoup *tw_fwd = nullptr;  // [M][N]: psi^brv(i)
    Shoup *tw_inv = nullptr;  // [M][N]: psi^-brv(i)
    uint64_t *twm_fwd = nullptr;  // [M][N]: tw_fwd's w 2^64 mod q (Montgomery form)
    uint64_t *twm_inv = nullptr;  // [M][N]: tw_inv's w 2^64 mod q
    ModC *mc = nullptr;       // [M]
    LastInv *li_plain = nullptr;  // [M]: scale 1
    LastInv *li_modup = nullptr;  // [L+1][L]: level l, limb i: scale (Qt_j/q_i)^-1 mod q_i
    LastInv *li_moddown = nullptr;  // [K]: scale (P/p_k)^-1 mod p_k
    uint64_t *conv_modup = nullptr;  // per level: [beta][l+K][alpha] of [Qt_j/q_i]_t (row j*E+t), split 25/25
    std::vector<size_t> conv_modup_off;  // [L+1]
    uint64_t *conv_moddown = nullptr;  // [L][K]: [P/p_k]_{q_i} (row i), split 25/25
    // ModDown by S = P q_(l-1) (NewMult at level l): special limbs p_0..p_(K-1), q_(l-1)
    LastInv *li_nm = nullptr;          // [L+1][K+1]: scale (S/s)^-1 mod s
    uint64_t *conv_nm = nullptr;       // per level: [l-1][K+1] of [S/s]_{q_i}, split 25/25
    std::vector<size_t> conv_nm_off;   // [L+1]
    Shoup *sinv_nm = nullptr;          // [L+1][L]: S^-1 mod q_i
    Shoup *pinv = nullptr;             // [L]: P^-1 mod q_i
    Shoup *pmod = nullptr;             // [L]: P mod q_i
    Shoup *rs_qinv = nullptr;          // [L+1][L]: q_{l-1}^-1 mod q_i
    uint64_t *rs_h = nullptr;          // [L+1][L]: ((q_{l-1}-1)/2) mod q_i
    uint32_t *enc_rotg = nullptr;      // [N/2]: 5^j mod 2N (the slots' rotation group)
    Cplx *enc_roots = nullptr;         // [2N]: exp(2 pi i t / 2N)
    LimbMap *dummy = nullptr;

    // workspace (device), sized for the top level and the batch capacity:
    // one slot per ciphertext of a batched key-switch step
    uint32_t batch_cap = 1;
    size_t ws_bytes = 0;
    uint64_t *ws = nullptr;
    uint64_t *ws_y = nullptr;    // [cap][L][N]          coefficient-form digits (ModUp)
    uint64_t *ws_ext = nullptr;  // [cap][dnum][L+K][N]  extended digits
    uint64_t *ws_uv = nullptr;   // [cap][2][L+K][N]     KSKInnerProd output on the q limbs
    uint64_t *ws_p = nullptr;    // [cap][2][K][N]       ModDown P-limbs (coefficient form)
    uint64_t *ws_z = nullptr;    // [cap][2][L][N]       ModDown correction
    uint64_t *ws_rot = nullptr;  // [cap][2][L][N]       PtMult / Mult output before Rescale
    uint64_t *ws_t = nullptr;    // [cap][3][L][N]       tensor product
    uint64_t *ws_r = nullptr;    // [2][N]               Rescale: coefficient-form last limbs
    uint64_t *ws_w = nullptr;    // [2][L][N]            Rescale: rounding correction
    size_t st_y() const { return (size_t)L * n; }
    size_t st_ext() const { return (size_t)dnum * M * n; }
    size_t st_uv() const { return (size_t)2 * M * n; }
    size_t st_p() const { return (size_t)2 * (K + 1) * n; }
    size_t st_z() const { return (size_t)2 * L * n; }
    size_t st_rot() const { return (size_t)2 * L * n; }
    size_t st_t() const { return (size_t)3 * L * n; }

    // kernel timing (hks_prof_*): event pairs per kernel class
    // canonical-range checks of call inputs (hks_set_check)
    bool check = false;
    uint32_t *chk_flag = nullptr;  // device word set by check_kernel
    mutable uint32_t prof_mask = 0;
    mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[HKS_K_COUNT];
    mutable std::vector<hipEvent_t> prof_pool;

    size_t ksk_words() const { return (size_t)dnum * 2 * M * n; }
};

// The workspace buffers one key-switch step uses, with the distance between
// the slots of consecutive batch entries: the context's own workspace, or
// the allocation-free scratch (hks_rotate_noalloc).
struct Ws {
    uint64_t *y, *ext, *uv, *p, *z;
    size_t st_y, st_ext, st_uv, st_p, st_z;  // words per batch entry (z: per polynomial)
};
inline Ws ctx_ws(const Ctx &c) {
    return Ws{c.ws_y, c.ws_ext, c.ws_uv, c.ws_p, c.ws_z, c.st_y(), c.st_ext(), c.st_uv(), c.st_p(), (size_t)c.L * c.n};
}

// Records a hipEvent pair around the launches in its scope when the class is
// selected by the context's timing mask.
struct ProfScope {
    const Ctx &c;
    int cls;
    hipStream_t s;
    bool on;
    ProfScope(const Ctx &ctx, int k, hipStream_t st);
    ~ProfScope();
};
void prof_reset(const Ctx &c);

// ---------------------------------------------------------------- tables (host)
int build_tables(Ctx &c);
void free_tables(Ctx &c);

// ---------------------------------------------------------------- launches (kernels.hip)
// All return hipSuccess or the launch error.
// NTT passes.  Every launcher runs the limbs of `m` for `batch` entries of
// `io` (in == out allowed).  Forward input residues < 2^53.
// Forward NTT, both passes; canonical output.
hipError_t launch_ntt_fwd(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s);
// Forward column pass only (lazy output for a row pass).
hipError_t launch_ntt_fwd_cols(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s);
// Forward row pass only (input: column-pass output); canonical output.
hipError_t launch_ntt_fwd_rows(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s);
// Inverse NTT, both passes, with the folded last stage li[cidx] (scale
// included); the row pass gathers entry b through the automorph
// io.galois[b] (1: none).  Canonical output.
hipError_t launch_ntt_inv(const Ctx &c, const LimbMap &m, const BatchIo &io, const LastInv *li, uint32_t batch,
                          hipStream_t s);
// Inverse row pass only (lazy output in [0, 2q)).
hipError_t launch_ntt_inv_rows(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s);
// Inverse column pass only, with the folded last stage li[cidx].
hipError_t launch_ntt_inv_cols(const Ctx &c, const LimbMap &m, const BatchIo &io, const LastInv *li,
                               uint32_t batch, hipStream_t s);
// Forward row pass of the ModDown correction z (io.in) followed by
// out = (u - z) * P^-1 (+ io.add gathered through io.add_galois).
hipError_t launch_rows_mdepi(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, const Shoup *pinv,
                             hipStream_t s);
// NewLimb of every digit of the coefficient-form y [level][N] into the other
// limbs of Q_level U P (coefficient form, canonical) for t outside digit j,
// for `batch` polynomials at strides y_bstride / ext_bstride, polynomial b at
// level levels[b].  Layout of the extended digits: packed, [beta][level + K]
// with limb t of digit j at j (level + K) + t; or key-indexed (keyidx),
// [beta][L + K] with the limb of modulus kappa (q_i: i, p_k: L + k) at
// j (L + K) + kappa, the same for every level.
hipError_t launch_conv_modup(const Ctx &c, const uint64_t *y, const uint32_t *levels, uint64_t *ext,
                             uint32_t batch, size_t y_bstride, size_t ext_bstride, bool keyidx, hipStream_t s);
// NewLimb of ModDown: the ns coefficient-form special limbs p [ns][N] (scaled
// by [(S/s)^-1]) into the nt[b] q limbs z [nt[b]][N] with constants table
// [nt][ns] of [S/s]_{q_i}, for `batch` polynomials.
hipError_t launch_conv_moddown(const Ctx &c, const uint64_t *p, const uint32_t *nt, uint64_t *z, uint32_t batch,
                               size_t p_bstride, size_t z_bstride, const uint64_t *table, uint32_t ns,
                               hipStream_t s);
// KSKInnerProd of `nb` ciphertexts per target limb and row tile (+ ModDown's
// inverse row pass for the P limbs).  Entry b is at level level[b]: its
// converted limb t of digit j at ext + b*ext_bstride + (j*E + t)*N (packed,
// E = level[b] + K) or at (j*(L+K) + kappa(t))*N (keyidx), after the forward
// column pass only (rowpass: the kernel runs the row pass) or in evaluation
// form; digit j's own limb (all digits if all_direct) at direct[b] +
// j*dstride + t*N, gathered through galois[b]; key ksk[b]; q limbs to uq +
// b*uq_bstride ([2][level[b]][N]), P limbs to pc + b*pc_bstride ([2][K][N]).
// With `seeded`, ksk[b] holds only the rows b_j ([dnum][L+K][N]) and the
// rows a_j are regenerated from seed[b] (Philox4x32-10, see seeded_key_a).
// With `newmult` (NewMult): P b3 and P c3 (b3 at addp[b], c3 at addp[b] +
// level N) are added to u and v on the q limbs, and q_(level-1) joins the
// special limbs (inverse row pass, stored after the P limbs).
struct KskBatch {
    const uint64_t *direct[MAXCT];
    const uint64_t *ksk[MAXCT];
    const uint64_t *addp[MAXCT];
    uint64_t seed[MAXCT];
    uint32_t galois[MAXCT];
    uint32_t level[MAXCT];
    uint32_t seeded;
    uint32_t newmult;
};
hipError_t launch_ksk_rows(const Ctx &c, const KskBatch &kb, uint32_t nb, const uint64_t *ext, size_t ext_bstride,
                           bool rowpass, bool keyidx, size_t dstride, uint32_t all_direct, uint64_t *uq,
                           size_t uq_bstride, uint64_t *pc, size_t pc_bstride, hipStream_t s);
// (the special limbs of one polynomial in pc: K, or K + 1 with newmult)
// PtMatVecMult sums over Q_level U P (ModUp'd digits of a in ext, evaluation
// form, [beta][level+K][N]): q limbs into uq [2][level][N], P limbs after
// ModDown's inverse row pass into pc [2][K][N].  r <= MAXROT.  ksk[i] ==
// nullptr (with galois[i] == 1) is the diagonal without rotation, read from
// the input's a (ax) and b.
hipError_t launch_ksk_matvec(const Ctx &c, const uint64_t *ext, uint32_t level, uint32_t r, const uint32_t *galois,
                             const uint64_t *const *ksk, const uint64_t *const *pt, const uint64_t *ax,
                             const uint64_t *b, uint64_t *uq, uint64_t *pc, hipStream_t s);
// Canonical-range check: sets *flag when a word of p, read as reps copies of
// `limbs` limbs with moduli first_mod.., is not below its modulus.
hipError_t launch_check(const Ctx &c, const uint64_t *p, uint32_t reps, uint32_t limbs, uint32_t first_mod,
                        uint32_t *flag, hipStream_t s);
hipError_t launch_clear_flag(uint32_t *flag, hipStream_t s);
// Independent lazy Shoup products into the workspace; *products = their count.
hipError_t launch_modmul_rate(const Ctx &c, uint32_t iters, hipStream_t s, uint64_t *products);
// The rows a_j of the seeded key `seed`: a [dnum][L+K][N].
hipError_t launch_expand_key_a(const Ctx &c, uint64_t seed, uint64_t *a, hipStream_t s);
// Eval-domain automorph (gather) of limbs; or coefficient-domain map with negation.
hipError_t launch_automorph(const Ctx &c, const LimbMap &m, const uint64_t *in, uint64_t *out,
                            uint32_t galois, int eval_domain, uint32_t batch, size_t in_bstride,
                            size_t out_bstride, hipStream_t s);
// KSKInnerProd over beta digits with optional automorph of ext (HRotate).
hipError_t launch_ksk(const Ctx &c, const uint64_t *ext, uint32_t level, uint32_t beta,
                      const uint64_t *ksk, uint64_t *uv, uint32_t galois, uint32_t batch,
                      size_t ext_bstride, size_t uv_bstride, hipStream_t s);
// Elementwise: out[l] = x[l] * y[l] mod q_l (pt mult) for n_poly polys of level limbs.
hipError_t launch_mulpt(const Ctx &c, const uint64_t *ct, const uint64_t *pt, uint64_t *out,
                        uint32_t level, uint32_t n_poly, hipStream_t s);
// Encoding, in two steps: x (N/2 complex) <- V^H x, bit-reversed (in place);
// then coefficients m = round(scale * (Re w, Im w)), w = V^H x / (N/2),
// reduced mod the limbs of m (out_off = limb of out, coefficient form,
// natural order).
hipError_t launch_enc_fft(const Ctx &c, Cplx *x, hipStream_t s);
hipError_t launch_enc_round(const Ctx &c, const Cplx *x, double scale, const LimbMap &m, uint64_t *out,
                            hipStream_t s);
// Tensor: (a1 a2, a1 b2 + a2 b1, b1 b2).
hipError_t launch_tensor(const Ctx &c, const uint64_t *ct1, const uint64_t *ct2, uint64_t *out3,
                         uint32_t level, hipStream_t s);
// out[l] = x[l] + y[l] mod q_l.
hipError_t launch_add(const Ctx &c, const uint64_t *x, const uint64_t *y, uint64_t *out,
                      uint32_t n_limbs_total, uint32_t level, hipStream_t s);
// Rescale tail: w_i = (r - h) mod q_i where r = coefficient-form last limb + h (mod q_last).
hipError_t launch_rescale_prep(const Ctx &c, const uint64_t *rlast, uint64_t *w, uint32_t level,
                               uint32_t n_poly, size_t r_bstride, size_t w_bstride, hipStream_t s);
// out_i = (x_i - w_i) * q_last^-1 mod q_i.
hipError_t launch_rescale_epi(const Ctx &c, const uint64_t *x, const uint64_t *w, uint64_t *out,
                              uint32_t level, uint32_t n_poly, size_t x_bstride, size_t w_bstride,
                              size_t out_bstride, hipStream_t s);
hipError_t launch_copy(const uint64_t *in, uint64_t *out, size_t words, hipStream_t s);

// ---------------------------------------------------------------- host math (tables.cpp)
uint64_t h_mulmod(uint64_t a, uint64_t b, uint64_t m);
uint64_t h_powmod(uint64_t a, uint64_t e, uint64_t m);
uint64_t h_invmod(uint64_t a, uint64_t m);
bool h_is_prime(uint64_t n);
uint64_t h_root_2n(uint64_t q, uint32_t log_n);
Shoup h_shoup(uint64_t w, uint64_t q);

}  // namespace hks

struct hks_ctx {
    hks::Ctx c;
};
