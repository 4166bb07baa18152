// Instantiations of the wavefront-per-shot decoder for lift size L = 16, H_X pattern.
#include "decode_wave.h"

namespace qldpc {

hipError_t launch_wavex_L16(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.which != 1) return hipErrorNotSupported;
    if (k.fmt == 0 && k.sched == 0) return launch_wave<ShapeLP35X, 16, 0, 0>(k, a, st);
    if (k.fmt == 0 && k.sched == 1) return launch_wave<ShapeLP35X, 16, 0, 1>(k, a, st);
    if (k.fmt == 1 && k.sched == 0) return launch_wave<ShapeLP35X, 16, 1, 0>(k, a, st);
    if (k.fmt == 1 && k.sched == 1) return launch_wave<ShapeLP35X, 16, 1, 1>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
