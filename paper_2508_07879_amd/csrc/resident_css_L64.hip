// Instantiations of the resident latency decoder for CSS pairs (H_Z and H_X
// syndromes of one code in one request) for lift size L = 64.
#include "decode_resident.h"

namespace qldpc {

hipError_t launch_resident_css_L64(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t st) {
    if (k.which != 2 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 0 && k.nw == 8) return launch_resident<ShapeLP35Z, 64, 0, 8, ShapeLP35X>(k, r, grid, st);
    if (k.fmt == 0 && k.nw == 16) return launch_resident<ShapeLP35Z, 64, 0, 16, ShapeLP35X>(k, r, grid, st);
    if (k.fmt == 1 && k.nw == 8) return launch_resident<ShapeLP35Z, 64, 1, 8, ShapeLP35X>(k, r, grid, st);
    if (k.fmt == 1 && k.nw == 16) return launch_resident<ShapeLP35Z, 64, 1, 16, ShapeLP35X>(k, r, grid, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
