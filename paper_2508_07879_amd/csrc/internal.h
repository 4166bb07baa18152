// Host-side internals shared by the C-ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qldpc.h"
#include "decode_generic_api.h"
#include "kernels.h"

namespace qldpc {

// Layout choice recorded by the autotuner.
struct TuneChoice {
    int layout = 0;   // QLDPC_LAYOUT_WAVE or QLDPC_LAYOUT_BLOCK
    int nw = 0;       // waves per shot for the block layout
    float ms = 0.f;   // measured time of the choice
};

// Batch size classes of the tuning table: 1, 2-64, 65-1024, 1025-16384, larger.
inline int size_class(int32_t batch) {
    if (batch <= 1) return 0;
    if (batch <= 64) return 1;
    if (batch <= 1024) return 2;
    if (batch <= 16384) return 3;
    return 4;
}

inline int tune_key(int fmt, int sched, int per_bit, int cls) {
    return ((fmt * 2 + sched) * 2 + per_bit) * 8 + cls;
}

qldpc_status set_error(qldpc_status st, const std::string &msg);
qldpc_status hip_error(hipError_t e, const char *what);

}  // namespace qldpc

struct qldpc_code_s {
    int32_t m = 0, n = 0, nnz = 0, max_dc = 0, max_dv = 0;
    int32_t L = 0, which = -1, device = 0;   // L = 0: no compiled block pattern (edge-list kernel)
    qldpc::DevCode *dev = nullptr;   // device copy of the shift tables (lifted codes)
    qldpc::GenCode gen{};            // device edge lists (codes without a compiled pattern)
    void *gen_mem = nullptr;         // the one allocation behind `gen`
    std::mutex tune_mu;
    std::map<int, qldpc::TuneChoice> tune;
};

namespace qldpc {

// Validates `p` against `code` and fills the launch key and kernel
// arguments for a decode of `batch` shots (buffers set by the caller).
qldpc_status prepare_decode(qldpc_code code, const qldpc_decode_params *p, int32_t batch, LaunchKey *key,
                            DecodeArgs *args);

// Launches the on-chip decoder that prepare_decode chose for `code`: the
// edge-list kernel for codes without a compiled block pattern, else the
// lifted kernels (launch_decode).
hipError_t launch_code_decode(qldpc_code code, const LaunchKey &k, const DecodeArgs &a, hipStream_t stream);

}  // namespace qldpc
