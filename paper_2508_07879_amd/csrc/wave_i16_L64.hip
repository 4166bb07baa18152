// Instantiations of the wavefront-per-shot decoder (messages in LDS) with
// int16 messages (Q8 priors) for L = 64, both block patterns.
#include "decode_wave.h"

namespace qldpc {

hipError_t launch_wave_i16_L64(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.fmt != 2) return hipErrorNotSupported;
    if (k.which == 0 && k.sched == 0) return launch_wave<ShapeLP35Z, 64, 2, 0>(k, a, st);
    if (k.which == 0 && k.sched == 1) return launch_wave<ShapeLP35Z, 64, 2, 1>(k, a, st);
    if (k.which == 1 && k.sched == 0) return launch_wave<ShapeLP35X, 64, 2, 0>(k, a, st);
    if (k.which == 1 && k.sched == 1) return launch_wave<ShapeLP35X, 64, 2, 1>(k, a, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
