// Instantiations of the resident latency decoder with int16 messages (Q8
// priors) for L = 64, both block patterns.
#include "decode_resident.h"

namespace qldpc {

hipError_t launch_resident_i16_L64(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t st) {
    if (k.fmt != 2 || k.sched != 0) return hipErrorNotSupported;
    if (k.which == 0 && k.nw == 8) return launch_resident<ShapeLP35Z, 64, 2, 8>(k, r, grid, st);
    if (k.which == 0 && k.nw == 16) return launch_resident<ShapeLP35Z, 64, 2, 16>(k, r, grid, st);
    if (k.which == 1 && k.nw == 8) return launch_resident<ShapeLP35X, 64, 2, 8>(k, r, grid, st);
    if (k.which == 1 && k.nw == 16) return launch_resident<ShapeLP35X, 64, 2, 16>(k, r, grid, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
