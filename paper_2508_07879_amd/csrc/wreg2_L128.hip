// Instantiations of the register-resident decoder with two wavefronts per shot
// for L = 128 (flooding; FP32, int8 and int16 messages; both block patterns).
#include "decode_wreg2.h"

namespace qldpc {

hipError_t launch_wreg2_L128(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.sched != 0 || k.L != 128) return hipErrorNotSupported;
    if (k.which == 0) {
        if (k.fmt == 0) return launch_wreg2<ShapeLP35Z, 0, 128>(k, a, st);
        if (k.fmt == 1) return launch_wreg2<ShapeLP35Z, 1, 128>(k, a, st);
        if (k.fmt == 2) return launch_wreg2<ShapeLP35Z, 2, 128>(k, a, st);
    } else if (k.which == 1) {
        if (k.fmt == 0) return launch_wreg2<ShapeLP35X, 0, 128>(k, a, st);
        if (k.fmt == 1) return launch_wreg2<ShapeLP35X, 1, 128>(k, a, st);
        if (k.fmt == 2) return launch_wreg2<ShapeLP35X, 2, 128>(k, a, st);
    }
    return hipErrorNotSupported;
}

}  // namespace qldpc
