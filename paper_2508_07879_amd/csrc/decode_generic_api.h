// Host-side interface of the edge-list decoder (codes given only as CSR,
// without a compiled quasi-cyclic block pattern).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace qldpc {

struct LaunchKey;
struct DecodeArgs;

// Device view of a code without lift data (one allocation per code object).
struct GenCode {
    int32_t m, n, nnz, max_dc;
    const int32_t *row_ptr;   // [m + 1]
    const int32_t *col_idx;   // [nnz], columns increasing per row
    const int32_t *col_ptr;   // [n + 1]
    const int32_t *vn_slot;   // [nnz]: j * m + r for the k-th edge of each variable, rows increasing
};

// LDS bytes of one wave: messages (max_dc * m entries), then the packed
// decisions and the packed syndrome, 16-byte aligned.
inline size_t gen_lds_bytes(int m, int n, int max_dc, int msg_bytes) {
    const size_t msg = ((size_t)max_dc * m * msg_bytes + 15) & ~size_t(15);
    return msg + 4 * (size_t)((n + 31) / 32) + 4 * (size_t)((m + 31) / 32);
}

// Most LDS one wavefront of the edge-list decoder may take.
constexpr size_t kGenMaxLds = 65536;

// Launches the edge-list decoder (flooding; format, prior mode and posterior
// from `k`) for a.batch shots; hipErrorNotSupported when the messages of the
// format do not fit kGenMaxLds.
hipError_t launch_generic_decode(const GenCode &g, const LaunchKey &k, const DecodeArgs &a, hipStream_t stream);

}  // namespace qldpc
