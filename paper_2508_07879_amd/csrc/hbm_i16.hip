// Instantiations of the HBM-message workgroup decoder with int16 messages
// (Q8 priors): lift sizes 128, 256, 512, both block patterns.
#include "decode_hbm.h"

namespace qldpc {

template <class S>
static hipError_t launch_hbm_i16_shape(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t st) {
    constexpr int NW = 8;
    switch (k.L) {
        case 128: return launch_hbm<S, 128, 2, NW>(k, a, ws, st);
        case 256: return launch_hbm<S, 256, 2, NW>(k, a, ws, st);
        case 512: return launch_hbm<S, 512, 2, NW>(k, a, ws, st);
        default: return hipErrorNotSupported;
    }
}

hipError_t launch_hbm_i16(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t st) {
    if (k.fmt != 2 || k.sched != 0) return hipErrorNotSupported;
    if (k.which == 0) return launch_hbm_i16_shape<ShapeLP35Z>(k, a, ws, st);
    if (k.which == 1) return launch_hbm_i16_shape<ShapeLP35X>(k, a, ws, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
