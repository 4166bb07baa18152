// Internal interface between the host runtime and the decoder kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qldpc {

constexpr int kMaxSlots = 120;   // block rows x check degree of the supported patterns

// Per-code device table (one allocation per code object).
constexpr int kMaxBlockCols = 34;   // block columns of the supported patterns
constexpr int kMaxColDeg = 5;       // nonzero blocks per block column

// Rotation data of one edge block, as the register-resident decoder reads it
// per block column (block rows increasing): the shift s, its complement
// c = (L - s) mod L, the byte offsets 4c and 4s of the cross-lane permutes
// (variable t meets check t - s = t + c mod L), and the low-bits mask of the
// segment rotation.
struct ColRot {
    int32_t s, c, c4, s4;
    uint64_t low;
    uint64_t pad;
};

// Per-code device table (one allocation per code object).
struct DevCode {
    int32_t shift[kMaxSlots];     // circulant shift of slot (R, j), in [0, L)
    uint64_t lowmask[kMaxSlots];  // L < 64: per-segment mask of the low L - shift bits
    ColRot colrot[kMaxBlockCols][kMaxColDeg];   // the same shifts by block column, L <= 64
};

// A DevCode seen through the constant address space.  No kernel writes the
// table; reading it this way makes the compiler fetch shifts with scalar
// loads, so that the rotations built from them run once per wave on the
// scalar unit.  The latency kernel, whose few waves per shot spend their
// time in those rotations, reads it so; the throughput kernels do not: in
// their hot loops the extra scalar loads cost more than the vector shifts
// they replace.
typedef const __attribute__((address_space(4))) DevCode *CodePtr;

__device__ __forceinline__ CodePtr const_code(const DevCode *p) { return (CodePtr)p; }

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
    const float *weights;   // neural decode: [weight_iters][nnz] per-edge scales
    int32_t weight_iters;   // neural decode: iterations 1..weight_iters use the weights, later ones alpha
};

// Doorbell page of a resident decoder, in mapped (fine-grained) host memory.
// The host writes `batch`, then `req_seq`; workgroup w of the resident grid
// answers by writing the served sequence number to done_seq[w] after its
// results are visible to the host.  `stop` asks the kernel to exit.
constexpr int kMaxResident = 64;   // shots per request of a resident session

struct ResidentRing {
    uint64_t req_seq;
    int32_t batch;
    int32_t stop;
    uint64_t pad[14];                  // done_seq starts on its own 128-byte line
    uint64_t done_seq[kMaxResident];
};

// Arguments of the resident decoder: `a` points its syndrome, prior and result
// buffers at mapped host staging; `cmd` is a device-memory mailbox
// [seq, batch] through which workgroup 0 relays requests to the others.
struct ResidentArgs {
    DecodeArgs a;
    const DevCode *code_x;  // CSS pair sessions: the H_X side's table (odd shots); else null
    ResidentRing *ring;
    uint64_t *cmd;
    uint64_t start_seq;    // last sequence number already served
    uint64_t idle_ticks;   // wall-clock ticks without a request before exiting
};

struct LaunchKey {
    int which;      // 0 = H_Z pattern, 1 = H_X pattern; 2 = a CSS pair (resident sessions)
    int L;          // 16, 32, 64, 128
    int fmt;        // 0 = F32, 1 = I8Q4, 2 = I16Q8
    int sched;      // 0 = flood, 1 = layered
    int per_bit;    // prior mode
    int post;       // posterior requested
    int layout;     // 1 = wave, 2 = block
    int nw;         // block layout: wavefronts per shot
};

// Returns hipErrorNotSupported when no kernel exists for the key.
hipError_t launch_decode(const LaunchKey &k, const DecodeArgs &a, hipStream_t stream);
// Launches the HBM-message workgroup decoder (layout 4) on workspace `ws`.
hipError_t launch_hbm_decode(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t stream);
// Launches the resident decoder (workgroup layout only) with `grid` shot slots.
hipError_t launch_resident_decode(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t stream);

}  // namespace qldpc
