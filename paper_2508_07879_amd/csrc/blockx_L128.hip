// Instantiations of the workgroup-per-shot decoder for lift size L = 128, H_X pattern.
#include "decode_block.h"

namespace qldpc {

hipError_t launch_blockx_L128(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which != 1 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 0 && k.nw == 8) return launch_block<ShapeLP35X, 128, 0, 8>(k, a, st);
    if (k.fmt == 0 && k.nw == 16) return launch_block<ShapeLP35X, 128, 0, 16>(k, a, st);
    if (k.fmt == 1 && k.nw == 8) return launch_block<ShapeLP35X, 128, 1, 8>(k, a, st);
    if (k.fmt == 1 && k.nw == 16) return launch_block<ShapeLP35X, 128, 1, 16>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
