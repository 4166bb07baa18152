// Internal interface between the host runtime and the decoder kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qldpc {

constexpr int kMaxSlots = 120;   // block rows x check degree of the supported patterns

// Per-code device table (one allocation per code object).
struct DevCode {
    int32_t shift[kMaxSlots];     // circulant shift of slot (R, j), in [0, L)
    uint64_t lowmask[kMaxSlots];  // L < 64: per-segment mask of the low L - shift bits
};

// Arguments shared by every decode kernel.
struct DecodeArgs {
    const DevCode *code;
    const uint32_t *syn;    // [batch][syn_words]
    const void *prior;      // float or int8, [batch] or [batch][n]
    uint32_t *err;          // [batch][err_words]
    uint8_t *conv;          // [batch]
    uint8_t *iters;         // [batch] or null
    float *post;            // [batch][n] or null
    int32_t batch;
    int32_t max_iters;
    int32_t early_stop;
    float alpha;            // F32
    int32_t alpha_num;      // I8Q4: alpha = alpha_num / 2^alpha_shift
    int32_t alpha_shift;
    const uint8_t *only;    // nullable: decode only shots with only[shot] != 0
    const float *weights;   // neural decode: [max_iters][nnz] per-edge scales
};

struct LaunchKey {
    int which;      // 0 = H_Z pattern, 1 = H_X pattern
    int L;          // 16, 32, 64, 128
    int fmt;        // 0 = F32, 1 = I8Q4
    int sched;      // 0 = flood, 1 = layered
    int per_bit;    // prior mode
    int post;       // posterior requested
    int layout;     // 1 = wave, 2 = block
    int nw;         // block layout: wavefronts per shot
};

// Returns hipErrorNotSupported when no kernel exists for the key.
hipError_t launch_decode(const LaunchKey &k, const DecodeArgs &a, hipStream_t stream);

}  // namespace qldpc
