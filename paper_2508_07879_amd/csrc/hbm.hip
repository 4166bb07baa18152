// Instantiations of the HBM-message workgroup decoder (lift sizes 128, 256,
// 512; both block patterns; FP32 and int8) and its launch (int16 in its own
// file).
#include "decode_hbm.h"

namespace qldpc {

constexpr int kHbmWaves = 8;

template <class S>
hipError_t launch_hbm_shape(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t st) {
    constexpr int NW = kHbmWaves;
    switch (k.L) {
        case 128: return k.fmt == 0 ? launch_hbm<S, 128, 0, NW>(k, a, ws, st) : launch_hbm<S, 128, 1, NW>(k, a, ws, st);
        case 256: return k.fmt == 0 ? launch_hbm<S, 256, 0, NW>(k, a, ws, st) : launch_hbm<S, 256, 1, NW>(k, a, ws, st);
        case 512: return k.fmt == 0 ? launch_hbm<S, 512, 0, NW>(k, a, ws, st) : launch_hbm<S, 512, 1, NW>(k, a, ws, st);
        default: return hipErrorNotSupported;
    }
}

hipError_t launch_hbm_i16(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t st);

hipError_t launch_hbm_decode(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t st) {
    if (k.layout != 4 || k.sched != 0) return hipErrorNotSupported;
    if (k.fmt == 2) return launch_hbm_i16(k, a, ws, st);
    if (k.fmt != 0 && k.fmt != 1) return hipErrorNotSupported;
    if (k.which == 0) return launch_hbm_shape<ShapeLP35Z>(k, a, ws, st);
    if (k.which == 1) return launch_hbm_shape<ShapeLP35X>(k, a, ws, st);
    return hipErrorNotSupported;
}

}  // namespace qldpc
