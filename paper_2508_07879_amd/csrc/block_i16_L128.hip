// Instantiations of the workgroup-per-shot decoder with int16 messages (Q8
// priors) for L = 128, both block patterns.
#include "decode_block.h"

namespace qldpc {

hipError_t launch_block_i16_L128(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.fmt != 2 || k.sched != 0) return hipErrorNotSupported;
    if (k.which == 0 && k.nw == 8) return launch_block<ShapeLP35Z, 128, 2, 8>(k, a, st);
    if (k.which == 0 && k.nw == 16) return launch_block<ShapeLP35Z, 128, 2, 16>(k, a, st);
    if (k.which == 1 && k.nw == 8) return launch_block<ShapeLP35X, 128, 2, 8>(k, a, st);
    if (k.which == 1 && k.nw == 16) return launch_block<ShapeLP35X, 128, 2, 16>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
