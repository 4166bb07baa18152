// Instantiations of the register-resident wavefront decoder for L = 32.
#include "decode_wave.h"

namespace qldpc {

hipError_t launch_wreg_L32(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which == 0) return launch_wreg<ShapeLP35Z, 32>(k, a, st);
    if (k.which == 1) return launch_wreg<ShapeLP35X, 32>(k, a, st);
    return hipErrorNotSupported;
}

hipError_t launch_wreg_weighted_L32(const DecodeArgs &a, hipStream_t st) {
    return launch_wreg_weighted<ShapeLP35Z, 32>(a, st);
}

}  // namespace qldpc
