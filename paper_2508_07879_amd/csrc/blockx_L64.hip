// Instantiations of the workgroup-per-shot decoder for lift size L = 64, H_X pattern.
#include "decode_block.h"

namespace qldpc {

hipError_t launch_blockx_L64(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which != 1 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 0 && k.nw == 8) return launch_block<ShapeLP35X, 64, 0, 8>(k, a, st);
    if (k.fmt == 0 && k.nw == 16) return launch_block<ShapeLP35X, 64, 0, 16>(k, a, st);
    if (k.fmt == 1 && k.nw == 8) return launch_block<ShapeLP35X, 64, 1, 8>(k, a, st);
    if (k.fmt == 1 && k.nw == 16) return launch_block<ShapeLP35X, 64, 1, 16>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
