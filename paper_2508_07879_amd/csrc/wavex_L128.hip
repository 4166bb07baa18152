// Instantiations of the wavefront-per-shot decoder for lift size L = 128, H_X pattern.
#include "decode_wave.h"

namespace qldpc {

hipError_t launch_wavex_L128(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which != 1) return hipErrorNotSupported;
    if (k.fmt == 0 && k.sched == 0) return launch_wave<ShapeLP35X, 128, 0, 0>(k, a, st);
    if (k.fmt == 0 && k.sched == 1) return launch_wave<ShapeLP35X, 128, 0, 1>(k, a, st);
    if (k.fmt == 1 && k.sched == 0) return launch_wave<ShapeLP35X, 128, 1, 0>(k, a, st);
    if (k.fmt == 1 && k.sched == 1) return launch_wave<ShapeLP35X, 128, 1, 1>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
