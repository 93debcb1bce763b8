// Host side of the NTT passes (Sec. 2.3): the launch sequence of a forward
// or inverse transform and the choice of each pass's launch shape from the
// context's plan.  The kernels are in ntt_device.h, instantiated by
// ntt_cols.hip, ntt_rows_fwd.hip and ntt_rows_inv.hip.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hks_internal.h"
#include "ntt_device.h"

namespace hks {

// Whether the entries of a launch sit at different levels (per-entry limb
// limits or constant offsets set): only then do its blocks test whether their
// entry has their limb.
static bool io_mixed(const BatchIo &io, uint32_t batch) {
    for (uint32_t b = 0; b < batch && b < (uint32_t)MAXB; ++b)
        if (io.lvl[b] || io.nbeta[b] || io.cbase[b]) return true;
    return false;
}

// Elements per thread: 16 (radix-16 phases) when the launch has enough
// waves to fill the chip several times over (the plan's threshold for the
// pass class: 6 waves per SIMD by default, never for the forward row pass
// by default), else 8 (radix-8 phases, one more LDS exchange, twice the
// waves with half the work each), so that a small launch still hides its
// memory latency.  Lines per block: the plan's column-tile width or rows per
// row tile for passes of 7 or more stages (the defaults for shorter ones, and
// when the plan's width would exceed 1024 threads per block).
template <bool COLS, bool FWD, int IO>
static hipError_t dispatch_pass(const NttArgs &a, int logs, uint32_t count, uint32_t batch, hipStream_t s) {
    if (count == 0 || batch == 0) return hipSuccess;
    if (batch > (uint32_t)MAXB) return hipErrorInvalidValue;
    int io = IO;
    if (io_mixed(a.io, batch)) {
        // the forward row pass with a reduced output serves whole transforms
        // (never a mixed-level step)
        if (IO == IO_REDUCE) return hipErrorInvalidValue;
        io |= IO_MIXED;
    }
    const hks_plan &p = a.ctx->plan;
    const uint64_t waves16 = (uint64_t)count * batch * ((1ull << a.n) / 16) / 64;
    const int cls = FWD ? (COLS ? HKS_K_NTT_FWD_COLS : HKS_K_NTT_FWD_ROWS)
                        : (COLS ? HKS_K_NTT_INV_COLS : HKS_K_NTT_INV_ROWS);
    const int e = waves16 >= p.e16_min_waves[cls] ? 16 : 8;
    int lines = COLS ? COL_LINES : ROW_LINES;
    if (logs >= 7) {
        const int want = COLS ? (int)p.col_lines : (int)p.row_lines;
        const int threads = want * ((1 << logs) / e);
        if (want && threads <= 1024 && (COLS || (1 << a.n1) >= want)) lines = want;
    }
    if (COLS) return launch_pass_cols(a, FWD, io, e, logs, lines, count, batch, s);
    return FWD ? launch_pass_rows_fwd(a, io, e, logs, lines, count, batch, s)
               : launch_pass_rows_inv(a, io, e, logs, lines, count, batch, s);
}

static NttArgs base_args(const Ctx &c, const LimbMap &m, const BatchIo &io, bool fwd) {
    NttArgs a{};
    a.ctx = &c;
    a.tw = fwd ? c.tw_fwd : c.tw_inv;
    a.twm = fwd ? c.twm_fwd : c.twm_inv;
    a.mc = c.mc;
    a.li = c.li_plain;
    a.pinv = c.pinv;
    a.n = c.log_n;
    a.n1 = c.n1;
    a.n2 = c.n2;
    a.L = c.L;
    a.m = m;
    a.io = io;
    return a;
}

// the second pass of a transform reads what the first wrote
static void chain(NttArgs &a, uint32_t batch) {
    for (uint32_t i = 0; i < a.m.count; ++i) a.m.in_off[i] = a.m.out_off[i];
    for (uint32_t b = 0; b < batch; ++b) {
        a.io.in[b] = a.io.out[b];
        a.io.galois[b] = 1;
    }
}

hipError_t launch_ntt_fwd(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    NttArgs a = base_args(c, m, io, true);
    hipError_t e = dispatch_pass<true, true, IO_PLAIN>(a, c.n1, m.count, batch, s);
    if (e != hipSuccess) return e;
    chain(a, batch);
    return dispatch_pass<false, true, IO_REDUCE>(a, c.n2, m.count, batch, s);
}

hipError_t launch_ntt_fwd_cols(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    return dispatch_pass<true, true, IO_PLAIN>(base_args(c, m, io, true), c.n1, m.count, batch, s);
}

hipError_t launch_ntt_fwd_rows(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    return dispatch_pass<false, true, IO_REDUCE>(base_args(c, m, io, true), c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv(const Ctx &c, const LimbMap &m, const BatchIo &io, const LastInv *li, uint32_t batch,
                          hipStream_t s) {
    NttArgs a = base_args(c, m, io, false);
    a.li = li;
    bool gather = false;
    for (uint32_t b = 0; b < batch && b < (uint32_t)MAXB; ++b) gather |= io.galois[b] != 1;
    hipError_t e = gather ? dispatch_pass<false, false, IO_GATHER>(a, c.n2, m.count, batch, s)
                          : dispatch_pass<false, false, IO_PLAIN>(a, c.n2, m.count, batch, s);
    if (e != hipSuccess) return e;
    chain(a, batch);
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

hipError_t launch_ntt_inv_rows(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, hipStream_t s) {
    return dispatch_pass<false, false, IO_PLAIN>(base_args(c, m, io, false), c.n2, m.count, batch, s);
}

hipError_t launch_ntt_inv_cols(const Ctx &c, const LimbMap &m, const BatchIo &io, const LastInv *li,
                               uint32_t batch, hipStream_t s) {
    NttArgs a = base_args(c, m, io, false);
    a.li = li;
    return dispatch_pass<true, false, IO_PLAIN>(a, c.n1, m.count, batch, s);
}

hipError_t launch_rows_mdepi(const Ctx &c, const LimbMap &m, const BatchIo &io, uint32_t batch, const Shoup *pinv,
                             hipStream_t s) {
    NttArgs a = base_args(c, m, io, true);
    a.pinv = pinv;
    return dispatch_pass<false, true, IO_MDEPI>(a, c.n2, m.count, batch, s);
}

}  // namespace hks
