// Instantiations of the resident latency decoder for lift size L = 64, H_X pattern.
#include "decode_resident.h"

namespace qldpc {

hipError_t launch_residentx_L64(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t st) {
    if (k.which != 1 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 0 && k.nw == 8) return launch_resident<ShapeLP35X, 64, 0, 8>(k, r, grid, st);
    if (k.fmt == 0 && k.nw == 16) return launch_resident<ShapeLP35X, 64, 0, 16>(k, r, grid, st);
    if (k.fmt == 1 && k.nw == 8) return launch_resident<ShapeLP35X, 64, 1, 8>(k, r, grid, st);
    if (k.fmt == 1 && k.nw == 16) return launch_resident<ShapeLP35X, 64, 1, 16>(k, r, grid, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
