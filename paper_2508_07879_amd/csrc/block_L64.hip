// Instantiations of the workgroup-per-shot decoder for lift size L = 64.
#include "decode_block.h"

namespace qldpc {

hipError_t launch_block_L64(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which != 0 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 0 && k.nw == 8) return launch_block<ShapeLP35Z, 64, 0, 8>(k, a, st);
    if (k.fmt == 0 && k.nw == 16) return launch_block<ShapeLP35Z, 64, 0, 16>(k, a, st);
    if (k.fmt == 1 && k.nw == 8) return launch_block<ShapeLP35Z, 64, 1, 8>(k, a, st);
    if (k.fmt == 1 && k.nw == 16) return launch_block<ShapeLP35Z, 64, 1, 16>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
