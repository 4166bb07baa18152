// Kernel selection for a decode call.
#include "kernels.h"

namespace qldpc {

hipError_t launch_wave_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_block_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_block_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_resident_L64(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_resident_L128(const LaunchKey &, const ResidentArgs &, int, hipStream_t);

hipError_t launch_decode(const LaunchKey &k, const DecodeArgs &a, hipStream_t stream) {
    if (k.layout == 1) {
        switch (k.L) {
            case 16: return launch_wave_L16(k, a, stream);
            case 32: return launch_wave_L32(k, a, stream);
            case 64: return launch_wave_L64(k, a, stream);
            case 128: return launch_wave_L128(k, a, stream);
            default: break;
        }
    }
    if (k.layout == 2) {
        if (k.L == 64) return launch_block_L64(k, a, stream);
        if (k.L == 128) return launch_block_L128(k, a, stream);
    }
    if (k.layout == 3) {
        switch (k.L) {
            case 16: return launch_wreg_L16(k, a, stream);
            case 32: return launch_wreg_L32(k, a, stream);
            case 64: return launch_wreg_L64(k, a, stream);
            default: break;
        }
    }
    return hipErrorNotSupported;
}

hipError_t launch_resident_decode(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t stream) {
    if (k.layout != 2) return hipErrorNotSupported;
    if (k.L == 64) return launch_resident_L64(k, r, grid, stream);
    if (k.L == 128) return launch_resident_L128(k, r, grid, stream);
    return hipErrorNotSupported;
}

}  // namespace qldpc
