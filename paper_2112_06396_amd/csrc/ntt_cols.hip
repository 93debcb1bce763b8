// Instantiations of the column passes (forward, and inverse with the folded
// last stage), uniform and mixed-level launches.
#include "pass_shapes.h"

namespace hks {

hipError_t launch_pass_cols(const NttArgs &a, bool fwd, int io, int e, int logs, int lines, uint32_t count,
                            uint32_t batch, hipStream_t s) {
    switch (io) {
        case IO_PLAIN:
            return fwd ? pass_by_e<true, true, IO_PLAIN>(a, e, logs, lines, count, batch, s)
                       : pass_by_e<true, false, IO_PLAIN>(a, e, logs, lines, count, batch, s);
        case IO_PLAIN | IO_MIXED:
            return fwd ? pass_by_e<true, true, IO_PLAIN | IO_MIXED>(a, e, logs, lines, count, batch, s)
                       : pass_by_e<true, false, IO_PLAIN | IO_MIXED>(a, e, logs, lines, count, batch, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace hks
