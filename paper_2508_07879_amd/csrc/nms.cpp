// C ABI of neural min-sum: per-edge, per-iteration weights in the check rule
// of flooding min-sum (Section 2, Algorithm 1 with alpha replaced by w[k][e]).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace qldpc {

struct NmsArgs;
hipError_t launch_nms_L32(int op, const NmsArgs &, const DecodeArgs &, hipStream_t);
hipError_t launch_nms_L64(int op, const NmsArgs &, const DecodeArgs &, hipStream_t);
hipError_t launch_nms_L128(int op, const NmsArgs &, const DecodeArgs &, hipStream_t);

}  // namespace qldpc

#include "decode_nms.h"

using namespace qldpc;

namespace {

constexpr int kMaxBwdWaves = 1024;

struct NmsGeom {
    int tiles, waves;
    size_t row, traj_floats, part_floats;
};

NmsGeom geom(qldpc_code c, int32_t batch, int32_t T) {
    NmsGeom g{};
    const int spw = c->L >= 64 ? 1 : 64 / c->L;
    g.row = (size_t)kMaxSlots * (c->L > 64 ? c->L : 64);
    g.tiles = (batch + spw - 1) / spw;
    g.waves = std::min(g.tiles, kMaxBwdWaves);
    g.traj_floats = (size_t)T * g.tiles * g.row;
    g.part_floats = (size_t)g.waves * T * g.row;
    return g;
}

hipError_t launch(qldpc_code c, int op, const NmsArgs &n, const DecodeArgs &d, hipStream_t st) {
    if (c->which != 0) return hipErrorNotSupported;
    switch (c->L) {
        case 32: return launch_nms_L32(op, n, d, st);
        case 64: return launch_nms_L64(op, n, d, st);
        case 128: return launch_nms_L128(op, n, d, st);
        default: return hipErrorNotSupported;
    }
}

qldpc_status check(qldpc_code c, int32_t batch, int32_t T) {
    if (!c) return set_error(QLDPC_ERR_INVALID_ARG, "nbp: null code");
    if (batch < 0) return set_error(QLDPC_ERR_INVALID_ARG, "nbp: negative batch");
    if (T < 1 || T > 255) return set_error(QLDPC_ERR_INVALID_ARG, "nbp: T must be in [1, 255]");
    if (c->which != 0 || (c->L != 32 && c->L != 64 && c->L != 128))
        return set_error(QLDPC_ERR_UNSUPPORTED, "nbp: neural kernels exist for H_Z patterns with L = 32, 64, 128");
    return QLDPC_OK;
}

qldpc_status result(hipError_t e, const char *what) {
    if (e == hipErrorNotSupported) return set_error(QLDPC_ERR_UNSUPPORTED, what);
    if (e != hipSuccess) return hip_error(e, what);
    return QLDPC_OK;
}

__global__ void k_zero(float *x, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

__global__ void k_not(const uint8_t *conv, uint8_t *out, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = conv[i] ? 0 : 1;
}
__global__ void k_beyond(const uint8_t *iters, int32_t T, uint8_t *out, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = iters[i] > T ? 1 : 0;
}

}  // namespace

extern "C" {

qldpc_status qldpc_nbp_workspace_bytes(qldpc_code code, int32_t batch, int32_t T, size_t *bytes) {
    qldpc_status st = check(code, batch, T);
    if (st != QLDPC_OK) return st;
    if (!bytes) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_workspace_bytes: null out");
    const NmsGeom g = geom(code, std::max(batch, 1), T);
    *bytes = (g.traj_floats + g.part_floats) * sizeof(float);
    return QLDPC_OK;
}

qldpc_status qldpc_nbp_forward(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                               const uint32_t *syn, const float *priors, float *posteriors, void *workspace,
                               void *stream) {
    qldpc_status st = check(code, batch, T);
    if (st != QLDPC_OK || batch == 0) return st;
    if (!weights || !syn || !priors || !posteriors || !workspace)
        return set_error(QLDPC_ERR_INVALID_ARG, "nbp_forward: null buffer");
    if (((uintptr_t)weights & 15) != 0) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_forward: weights must be 16-byte aligned");
    const NmsGeom g = geom(code, batch, T);
    NmsArgs n{};
    n.code = code->dev;
    n.syn = syn;
    n.prior = priors;
    n.w = weights;
    n.post = posteriors;
    n.traj = static_cast<float *>(workspace);
    n.partial = n.traj + g.traj_floats;
    n.batch = batch;
    n.T = T;
    n.tiles = g.tiles;
    n.waves = g.waves;
    return result(launch(code, 0, n, DecodeArgs{}, (hipStream_t)stream), "nbp_forward");
}

qldpc_status qldpc_nbp_backward(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                                const uint32_t *syn, const void *workspace, const float *grad_posteriors,
                                float *grad_weights, void *stream) {
    qldpc_status st = check(code, batch, T);
    if (st != QLDPC_OK) return st;
    if (!weights || !grad_weights) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_backward: null buffer");
    if (batch == 0) {
        const size_t n = (size_t)T * code->nnz;
        hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, grad_weights, n);
        return result(hipGetLastError(), "nbp_backward: clear");
    }
    if (!syn || !workspace || !grad_posteriors) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_backward: null buffer");
    if (((uintptr_t)weights & 15) != 0) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_backward: weights must be 16-byte aligned");
    const NmsGeom g = geom(code, batch, T);
    NmsArgs n{};
    n.code = code->dev;
    n.syn = syn;
    n.w = weights;
    n.gpost = grad_posteriors;
    n.traj = const_cast<float *>(static_cast<const float *>(workspace));
    n.partial = n.traj + g.traj_floats;
    n.grad_w = grad_weights;
    n.batch = batch;
    n.T = T;
    n.tiles = g.tiles;
    n.waves = g.waves;
    st = result(launch(code, 1, n, DecodeArgs{}, (hipStream_t)stream), "nbp_backward");
    if (st != QLDPC_OK) return st;
    return result(launch(code, 2, n, DecodeArgs{}, (hipStream_t)stream), "nbp_backward: reduce");
}

qldpc_status qldpc_nbp_decode(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                              const qldpc_decode_params *fallback, const uint32_t *syn, const float *priors,
                              uint32_t *errors, uint8_t *converged, uint8_t *iters_used, uint8_t *used_fallback,
                              void *stream) {
    qldpc_status st = check(code, batch, T);
    if (st != QLDPC_OK || batch == 0) return st;
    if (!weights || !syn || !priors || !errors || !converged || !used_fallback)
        return set_error(QLDPC_ERR_INVALID_ARG, "nbp_decode: null buffer");
    if (((uintptr_t)weights & 15) != 0) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_decode: weights must be 16-byte aligned");
    if (fallback && (fallback->fmt != QLDPC_F32 || fallback->prior_mode != QLDPC_PRIOR_PER_SHOT))
        return set_error(QLDPC_ERR_UNSUPPORTED, "nbp_decode: the fallback decodes FP32 with per-shot priors");
    hipStream_t s = (hipStream_t)stream;
    // pass 1: neural min-sum with early stop, at most T iterations
    DecodeArgs d{};
    d.code = code->dev;
    d.syn = syn;
    d.prior = priors;
    d.err = errors;
    d.conv = converged;
    d.iters = iters_used;
    d.batch = batch;
    d.max_iters = T;
    d.early_stop = 1;
    d.alpha = 1.0f;
    d.weights = weights;
    d.weight_iters = T;
    st = result(launch(code, 3, NmsArgs{}, d, s), "nbp_decode: neural pass");
    if (st != QLDPC_OK) return st;
    hipLaunchKernelGGL(k_not, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, converged, used_fallback, batch);
    st = result(hipGetLastError(), "nbp_decode: mark");
    if (st != QLDPC_OK || !fallback) return st;
    // pass 2: plain min-sum from scratch on the shots that did not converge
    LaunchKey k{};
    DecodeArgs f{};
    st = prepare_decode(code, fallback, batch, &k, &f);
    if (st != QLDPC_OK) return st;
    f.syn = syn;
    f.prior = priors;
    f.err = errors;
    f.conv = converged;
    f.iters = iters_used;
    f.only = used_fallback;
    k.post = 0;
    return result(launch_decode(k, f, s), "nbp_decode: fallback pass");
}

qldpc_status qldpc_nbp_decode_continue(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                                       int32_t max_iters, float alpha, const uint32_t *syn, const float *priors,
                                       uint32_t *errors, uint8_t *converged, uint8_t *iters_used,
                                       uint8_t *used_fallback, void *stream) {
    qldpc_status st = check(code, batch, T);
    if (st != QLDPC_OK || batch == 0) return st;
    if (max_iters < T || max_iters > 255)
        return set_error(QLDPC_ERR_INVALID_ARG, "nbp_decode_continue: max_iters must be in [T, 255]");
    if (!(alpha > 0.0f && alpha <= 1.0f)) return set_error(QLDPC_ERR_INVALID_ARG, "nbp_decode_continue: alpha must be in (0, 1]");
    if (!weights || !syn || !priors || !errors || !converged || !iters_used || !used_fallback)
        return set_error(QLDPC_ERR_INVALID_ARG, "nbp_decode_continue: null buffer");
    if (((uintptr_t)weights & 15) != 0)
        return set_error(QLDPC_ERR_INVALID_ARG, "nbp_decode_continue: weights must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    // one pass: weights in iterations 1..T, alpha after, early stop throughout
    DecodeArgs d{};
    d.code = code->dev;
    d.syn = syn;
    d.prior = priors;
    d.err = errors;
    d.conv = converged;
    d.iters = iters_used;
    d.batch = batch;
    d.max_iters = max_iters;
    d.early_stop = 1;
    d.alpha = alpha;
    d.weights = weights;
    d.weight_iters = T;
    st = result(launch(code, 3, NmsArgs{}, d, s), "nbp_decode_continue");
    if (st != QLDPC_OK) return st;
    hipLaunchKernelGGL(k_beyond, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, iters_used, T, used_fallback,
                       batch);
    return result(hipGetLastError(), "nbp_decode_continue: mark");
}

}  // extern "C"
