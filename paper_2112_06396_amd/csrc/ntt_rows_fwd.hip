// Instantiations of the forward row passes: with a reduced output (the last
// pass of a transform) and with ModDown's epilogue (uniform and mixed-level).
#include "pass_shapes.h"

namespace hks {

hipError_t launch_pass_rows_fwd(const NttArgs &a, int io, int e, int logs, int lines, uint32_t count,
                                uint32_t batch, hipStream_t s) {
    switch (io) {
        case IO_REDUCE: return pass_by_e<false, true, IO_REDUCE>(a, e, logs, lines, count, batch, s);
        case IO_MDEPI: return pass_by_e<false, true, IO_MDEPI>(a, e, logs, lines, count, batch, s);
        case IO_MDEPI | IO_MIXED: return pass_by_e<false, true, IO_MDEPI | IO_MIXED>(a, e, logs, lines, count, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hks
