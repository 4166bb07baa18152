// Instantiations of the resident latency decoder for lift size L = 128, H_X pattern.
#include "decode_resident.h"

namespace qldpc {

hipError_t launch_residentx_L128(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t st) {
    if (k.which != 1 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 0 && k.nw == 8) return launch_resident<ShapeLP35X, 128, 0, 8>(k, r, grid, st);
    if (k.fmt == 0 && k.nw == 16) return launch_resident<ShapeLP35X, 128, 0, 16>(k, r, grid, st);
    if (k.fmt == 1 && k.nw == 8) return launch_resident<ShapeLP35X, 128, 1, 8>(k, r, grid, st);
    if (k.fmt == 1 && k.nw == 16) return launch_resident<ShapeLP35X, 128, 1, 16>(k, r, grid, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
