// Run-time selection of a pass kernel by launch shape (included by the
// files that instantiate the pass kernels).
#pragma once
#include "ntt_device.h"

namespace hks {

// logs 5..9 stages; passes of 7 or more stages in three widths (lines per
// block), shorter ones in the default width only.
template <bool COLS, bool FWD, int IO, int E>
static hipError_t pass_by_shape(const NttArgs &a, int logs, int lines, uint32_t count, uint32_t batch,
                                hipStream_t s) {
    constexpr int D = COLS ? COL_LINES : ROW_LINES;
    constexpr int NARROW = D / 2, WIDE = D * 2;
#define HKS_PASS_LINES(LG)                                                                        \
    if (lines == NARROW) return launch_pass_t<LG, COLS, FWD, IO, E, NARROW>(a, count, batch, s); \
    if (lines == D) return launch_pass_t<LG, COLS, FWD, IO, E, D>(a, count, batch, s);           \
    if (lines == WIDE) return launch_pass_t<LG, COLS, FWD, IO, E, WIDE>(a, count, batch, s);     \
    return hipErrorInvalidValue;
    switch (logs) {
        case 5: return lines == D ? launch_pass_t<5, COLS, FWD, IO, E, D>(a, count, batch, s) : hipErrorInvalidValue;
        case 6: return lines == D ? launch_pass_t<6, COLS, FWD, IO, E, D>(a, count, batch, s) : hipErrorInvalidValue;
        case 7: { HKS_PASS_LINES(7) }
        case 8: { HKS_PASS_LINES(8) }
        case 9: { HKS_PASS_LINES(9) }
        default: return hipErrorInvalidValue;
    }
#undef HKS_PASS_LINES
}

template <bool COLS, bool FWD, int IO>
static hipError_t pass_by_e(const NttArgs &a, int e, int logs, int lines, uint32_t count, uint32_t batch,
                            hipStream_t s) {
    return e == 16 ? pass_by_shape<COLS, FWD, IO, 16>(a, logs, lines, count, batch, s)
                   : pass_by_shape<COLS, FWD, IO, 8>(a, logs, lines, count, batch, s);
}

}  // namespace hks
