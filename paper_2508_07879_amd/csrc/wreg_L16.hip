// Instantiations of the register-resident wavefront decoder for L = 16.
#include "decode_wave.h"

namespace qldpc {

hipError_t launch_wreg_L16(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which == 0) return launch_wreg<ShapeLP35Z, 16>(k, a, st);
    if (k.which == 1) return launch_wreg<ShapeLP35X, 16>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
