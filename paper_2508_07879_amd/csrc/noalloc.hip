// qldpc_decode_batch_static: qldpc_decode_batch_ws with the message
// workspace taken from a device buffer the library owns, for callers that
// cannot allocate device memory.
//
// The buffer is a file-scope __device__ array, so each GPU the library runs
// on holds its own copy for the life of the process.  Host code never uses
// the array's name as a device address: on the first call on a device, with
// that device current, its address is looked up once (hipGetSymbolAddress)
// and kept per device; kernels receive that address as their workspace
// argument, exactly as they receive a caller's workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

constexpr size_t kStaticBytes = QLDPC_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (resolved on first use, with `device`
// current); null with the error recorded on failure.
qldpc_status scratch_of(int device, void **out) {
    if (device < 0 || device >= kMaxDevices)
        return qldpc::set_error(QLDPC_ERR_INVALID_ARG, "decode_batch_static: device index out of range");
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_ptr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return qldpc::hip_error(e, "decode_batch_static: hipGetDevice");
        e = hipSetDevice(device);
        if (e != hipSuccess) return qldpc::hip_error(e, "decode_batch_static: hipSetDevice");
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(prev);
        if (e != hipSuccess) return qldpc::hip_error(e, "decode_batch_static: hipGetSymbolAddress");
        if (e2 != hipSuccess) return qldpc::hip_error(e2, "decode_batch_static: hipSetDevice");
        if (!p || ((uintptr_t)p & 255) != 0)
            return qldpc::set_error(QLDPC_ERR_DEVICE, "decode_batch_static: static workspace address unusable");
        g_ptr[device] = p;
    }
    *out = g_ptr[device];
    return QLDPC_OK;
}

}  // namespace

extern "C" {

qldpc_status qldpc_decode_batch_static(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                                       const uint32_t *syndromes, const void *priors, uint32_t *errors,
                                       uint8_t *converged, uint8_t *iters_used, float *posterior, void *stream) {
    if (!code) return qldpc::set_error(QLDPC_ERR_INVALID_ARG, "decode_batch_static: null code");
    size_t need = 0;
    qldpc_status st = qldpc_decode_workspace_bytes(code, params, batch, &need);
    if (st != QLDPC_OK) return st;
    if (need > kStaticBytes)
        return qldpc::set_error(QLDPC_ERR_CAPACITY,
                                "decode_batch_static: the batch needs " + std::to_string(need) +
                                    " bytes of message workspace; the static workspace holds " +
                                    std::to_string(kStaticBytes) + " (decode fewer shots per call)");
    void *ws = nullptr;
    if (need > 0) {
        st = scratch_of(code->device, &ws);
        if (st != QLDPC_OK) return st;
    }
    return qldpc_decode_batch_ws(code, params, batch, syndromes, priors, errors, converged, iters_used, posterior,
                                 ws, kStaticBytes, stream);
}

}  // extern "C"
