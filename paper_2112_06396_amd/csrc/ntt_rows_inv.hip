// Instantiations of the inverse row passes: plain and with the automorphism
// gathered in the loads (uniform and mixed-level).
#include "pass_shapes.h"

namespace hks {

hipError_t launch_pass_rows_inv(const NttArgs &a, int io, int e, int logs, int lines, uint32_t count,
                                uint32_t batch, hipStream_t s) {
    switch (io) {
        case IO_PLAIN: return pass_by_e<false, false, IO_PLAIN>(a, e, logs, lines, count, batch, s);
        case IO_PLAIN | IO_MIXED: return pass_by_e<false, false, IO_PLAIN | IO_MIXED>(a, e, logs, lines, count, batch, s);
        case IO_GATHER: return pass_by_e<false, false, IO_GATHER>(a, e, logs, lines, count, batch, s);
        case IO_GATHER | IO_MIXED:
            return pass_by_e<false, false, IO_GATHER | IO_MIXED>(a, e, logs, lines, count, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hks
