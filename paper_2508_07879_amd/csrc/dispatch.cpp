// Kernel selection for a decode call: layout, lift size and block pattern
// (which = 0: H_Z, 1: H_X).
#include "kernels.h"

namespace qldpc {

hipError_t launch_wave_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wavex_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wavex_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wavex_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wavex_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_block_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_block_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_blockx_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_blockx_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg2_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg2_L256(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg2_L512(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_i16_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_i16_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_i16_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wave_i16_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_block_i16_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_block_i16_L128(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_i16_L16(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_i16_L32(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_wreg_i16_L64(const LaunchKey &, const DecodeArgs &, hipStream_t);
hipError_t launch_resident_i16_L64(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_resident_i16_L128(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_resident_css_L64(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_resident_css_L128(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_resident_L64(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_resident_L128(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_residentx_L64(const LaunchKey &, const ResidentArgs &, int, hipStream_t);
hipError_t launch_residentx_L128(const LaunchKey &, const ResidentArgs &, int, hipStream_t);

// int16 messages: one set of files per layout, covering both patterns.
static hipError_t launch_decode_i16(const LaunchKey &k, const DecodeArgs &a, hipStream_t stream) {
    if (k.layout == 1) {
        switch (k.L) {
            case 16: return launch_wave_i16_L16(k, a, stream);
            case 32: return launch_wave_i16_L32(k, a, stream);
            case 64: return launch_wave_i16_L64(k, a, stream);
            case 128: return launch_wave_i16_L128(k, a, stream);
            default: break;
        }
    }
    if (k.layout == 2) {
        if (k.L == 64) return launch_block_i16_L64(k, a, stream);
        if (k.L == 128) return launch_block_i16_L128(k, a, stream);
    }
    if (k.layout == 3) {
        switch (k.L) {
            case 16: return launch_wreg_i16_L16(k, a, stream);
            case 32: return launch_wreg_i16_L32(k, a, stream);
            case 64: return launch_wreg_i16_L64(k, a, stream);
            case 128: return launch_wreg2_L128(k, a, stream);
            case 256: return launch_wreg2_L256(k, a, stream);
            case 512: return launch_wreg2_L512(k, a, stream);
            default: break;
        }
    }
    return hipErrorNotSupported;
}

hipError_t launch_decode(const LaunchKey &k, const DecodeArgs &a, hipStream_t stream) {
    const bool x = k.which == 1;
    if (k.which != 0 && k.which != 1) return hipErrorNotSupported;
    if (k.fmt == 2) return launch_decode_i16(k, a, stream);
    if (k.fmt != 0 && k.fmt != 1) return hipErrorNotSupported;
    if (k.layout == 1) {
        switch (k.L) {
            case 16: return x ? launch_wavex_L16(k, a, stream) : launch_wave_L16(k, a, stream);
            case 32: return x ? launch_wavex_L32(k, a, stream) : launch_wave_L32(k, a, stream);
            case 64: return x ? launch_wavex_L64(k, a, stream) : launch_wave_L64(k, a, stream);
            case 128: return x ? launch_wavex_L128(k, a, stream) : launch_wave_L128(k, a, stream);
            default: break;
        }
    }
    if (k.layout == 2) {
        if (k.L == 64) return x ? launch_blockx_L64(k, a, stream) : launch_block_L64(k, a, stream);
        if (k.L == 128) return x ? launch_blockx_L128(k, a, stream) : launch_block_L128(k, a, stream);
    }
    if (k.layout == 3) {
        switch (k.L) {
            case 16: return launch_wreg_L16(k, a, stream);
            case 32: return launch_wreg_L32(k, a, stream);
            case 64: return launch_wreg_L64(k, a, stream);
            case 128: return launch_wreg2_L128(k, a, stream);
            case 256: return launch_wreg2_L256(k, a, stream);
            case 512: return launch_wreg2_L512(k, a, stream);
            default: break;
        }
    }
    return hipErrorNotSupported;
}

hipError_t launch_resident_decode(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t stream) {
    if (k.layout != 2) return hipErrorNotSupported;
    if (k.which == 2) {   // CSS pair: FP32 and int8
        if (k.L == 64) return launch_resident_css_L64(k, r, grid, stream);
        if (k.L == 128) return launch_resident_css_L128(k, r, grid, stream);
        return hipErrorNotSupported;
    }
    if (k.fmt == 2) {
        if (k.L == 64) return launch_resident_i16_L64(k, r, grid, stream);
        if (k.L == 128) return launch_resident_i16_L128(k, r, grid, stream);
        return hipErrorNotSupported;
    }
    const bool x = k.which == 1;
    if (k.L == 64) return x ? launch_residentx_L64(k, r, grid, stream) : launch_resident_L64(k, r, grid, stream);
    if (k.L == 128) return x ? launch_residentx_L128(k, r, grid, stream) : launch_resident_L128(k, r, grid, stream);
    return hipErrorNotSupported;
}

}  // namespace qldpc
