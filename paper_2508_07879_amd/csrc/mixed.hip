// Mixed-code persistent decoder: launch sequence and C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "decode_mixed.h"
#include "internal.h"

using namespace qldpc;

struct qldpc_mixed_s {
    int32_t ncodes = 0, max_batch = 0, use_graph = 0, device = 0;
    qldpc_code codes[kMaxMixCodes] = {};
    qldpc_decode_params params{};
    int32_t waves = 0;              // persistent grid size for each lift L <= 64 (registers)
    int32_t waves128 = 0;           // two-wave workgroups of the L = 128 grid
    bool has_grid[mix::kMixGrids] = {};   // (pattern, L) pairs among the plan's codes
    int32_t *scratch = nullptr;     // device
    // Captured plans run the grids of each lift size on a stream of their
    // own, forked from and joined back into the capture stream: they become
    // parallel graph branches, so a grid's tail is filled by the waves of the
    // others instead of the next grid waiting for it.  Eager plans (several
    // of which a server runs at once, one per slot, on a few hardware
    // queues) use one side stream for the L = 128 grids and run the others
    // one after the other on the caller's stream.
    static constexpr int kBranches = 4;   // lifts 128, 64, 32, 16
    int nside() const { return use_graph ? kBranches : 1; }
    hipStream_t side[kBranches] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kBranches] = {};
    std::mutex mu;
    std::map<std::tuple<int32_t, const void *, const void *, const void *, const void *, const void *, const void *,
                        const void *, const void *, const void *, void *, int32_t>,
             hipGraphExec_t>
        graphs;
};

namespace {

qldpc_status enqueue(qldpc_mixed x, int32_t batch, const int32_t *shot_code, const int64_t *syn_off,
                     const int64_t *err_off, const uint32_t *syn, const float *prior, uint32_t *err, uint8_t *conv,
                     uint8_t *iters, hipStream_t st, int32_t waves) {
    MixedArgs m{};
    m.base.alpha = x->params.alpha;
    m.base.max_iters = x->params.max_iters;
    m.base.early_stop = x->params.early_stop ? 1 : 0;
    m.base.prior = prior;
    m.base.conv = conv;
    m.base.iters = iters;
    m.base.batch = batch;
    m.ncodes = x->ncodes;
    for (int c = 0; c < x->ncodes; ++c) {
        m.codes[c] = x->codes[c]->dev;
        m.L[c] = x->codes[c]->L;
        m.which[c] = x->codes[c]->which;
    }
    // bucket order: largest L first, then code index
    for (int c = 0; c < x->ncodes; ++c) {
        int r = 0;
        for (int d = 0; d < x->ncodes; ++d)
            if (m.L[d] > m.L[c] || (m.L[d] == m.L[c] && d < c)) ++r;
        m.rank[c] = r;
    }
    m.shot_code = shot_code;
    m.syn_off = syn_off;
    m.err_off = err_off;
    m.syn = syn;
    m.err = err;
    m.scratch = x->scratch;
    m.batch = batch;
    // bucketing: at most 256 workgroups of 1024 threads, grid-stride over the shots
    const unsigned nb = (unsigned)std::min<int64_t>(256, (batch + kBucketThreads - 1) / kBucketThreads);
    hipLaunchKernelGGL(k_mix_clear, dim3(1), dim3(64), 0, st, m);
    hipLaunchKernelGGL(k_mix_count, dim3(nb), dim3(kBucketThreads), 0, st, m);
    hipLaunchKernelGGL(k_mix_plan, dim3(1), dim3(64), 0, st, m);
    hipLaunchKernelGGL(k_mix_scatter, dim3(nb), dim3(kBucketThreads), 0, st, m);
    // one persistent grid per (pattern, lift size) present, largest L first,
    // each lift size on its own branch when there are several
    const unsigned w64 = (unsigned)waves, w128 = (unsigned)x->waves128;
    const bool *g = x->has_grid;
    const bool lift[qldpc_mixed_s::kBranches] = {g[3] || g[7], g[2] || g[6], g[1] || g[5], g[0] || g[4]};
    const int nlift = (int)lift[0] + (int)lift[1] + (int)lift[2] + (int)lift[3];
    const bool fork = nlift > 1 && (x->use_graph || lift[0]);
    hipError_t fe = hipSuccess;
    if (fork && (fe = hipEventRecord(x->ev_fork, st)) != hipSuccess) return hip_error(fe, "mixed_decode: fork");
    for (int b = 0; b < qldpc_mixed_s::kBranches; ++b) {
        if (!lift[b]) continue;
        const bool own = fork && b < x->nside();   // this lift on a side stream
        hipStream_t bs = st;
        if (own) {
            if ((fe = hipStreamWaitEvent(x->side[b], x->ev_fork, 0)) != hipSuccess)
                return hip_error(fe, "mixed_decode: fork");
            bs = x->side[b];
        }
        switch (b) {
            case 0:
                if (g[3]) hipLaunchKernelGGL((k_mix_wreg2<ShapeLP35Z>), dim3(w128), dim3(128), 0, bs, m);
                if (g[7]) hipLaunchKernelGGL((k_mix_wreg2<ShapeLP35X>), dim3(w128), dim3(128), 0, bs, m);
                break;
            case 1:
                if (g[2]) hipLaunchKernelGGL((k_mix_decode<ShapeLP35Z, 64>), dim3(w64), dim3(64), 0, bs, m);
                if (g[6]) hipLaunchKernelGGL((k_mix_decode<ShapeLP35X, 64>), dim3(w64), dim3(64), 0, bs, m);
                break;
            case 2:
                if (g[1]) hipLaunchKernelGGL((k_mix_decode<ShapeLP35Z, 32>), dim3(w64), dim3(64), 0, bs, m);
                if (g[5]) hipLaunchKernelGGL((k_mix_decode<ShapeLP35X, 32>), dim3(w64), dim3(64), 0, bs, m);
                break;
            default:
                if (g[0]) hipLaunchKernelGGL((k_mix_decode<ShapeLP35Z, 16>), dim3(w64), dim3(64), 0, bs, m);
                if (g[4]) hipLaunchKernelGGL((k_mix_decode<ShapeLP35X, 16>), dim3(w64), dim3(64), 0, bs, m);
                break;
        }
        if (own && (fe = hipEventRecord(x->ev_join[b], x->side[b])) != hipSuccess)
            return hip_error(fe, "mixed_decode: join");
    }
    // the caller's stream waits for the side branches only after its own
    // grids are enqueued, so those run beside them
    for (int b = 0; b < qldpc_mixed_s::kBranches; ++b)
        if (lift[b] && fork && b < x->nside() && (fe = hipStreamWaitEvent(st, x->ev_join[b], 0)) != hipSuccess)
            return hip_error(fe, "mixed_decode: join");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "mixed_decode: launch");
    return QLDPC_OK;
}

}  // namespace

extern "C" {

qldpc_status qldpc_mixed_create(const qldpc_code *codes, int32_t ncodes, const qldpc_decode_params *params,
                                int32_t max_batch, int32_t use_graph, qldpc_mixed *out) {
    if (!codes || !params || !out) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_create: null argument");
    if (ncodes < 1 || ncodes > kMaxMixCodes) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_create: 1 to 8 codes");
    if (max_batch < 1) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_create: max_batch must be positive");
    if (params->fmt != QLDPC_F32 || params->sched != QLDPC_FLOOD || params->prior_mode != QLDPC_PRIOR_PER_SHOT)
        return set_error(QLDPC_ERR_UNSUPPORTED, "mixed_create: FP32 flooding with per-shot priors only");
    if (params->max_iters < 1 || params->max_iters > 255 || !(params->alpha > 0.f && params->alpha <= 1.f))
        return set_error(QLDPC_ERR_INVALID_ARG, "mixed_create: bad iterations or alpha");
    for (int c = 0; c < ncodes; ++c) {
        if (!codes[c]) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_create: null code");
        if (codes[c]->device != codes[0]->device) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_create: codes on different devices");
    }
    auto *x = new (std::nothrow) qldpc_mixed_s();
    if (!x) return set_error(QLDPC_ERR_OUT_OF_MEMORY, "mixed_create: host allocation");
    x->ncodes = ncodes;
    x->max_batch = max_batch;
    x->use_graph = use_graph ? 1 : 0;
    x->device = codes[0]->device;
    std::copy(codes, codes + ncodes, x->codes);
    x->params = *params;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, x->device);
    x->waves = 12 * cus;     // register grids: up to three waves per SIMD
    x->waves128 = 6 * cus;   // L = 128: six two-wave workgroups per CU (three waves per SIMD)
    for (int c = 0; c < ncodes; ++c) {
        const int L = codes[c]->L;
        if (L != 16 && L != 32 && L != 64 && L != 128) {
            delete x;
            return set_error(QLDPC_ERR_UNSUPPORTED, "mixed_create: lifts 16, 32, 64 and 128 only");
        }
        x->has_grid[mix::grid_of(codes[c]->which, L)] = true;
    }
    hipError_t e = hipSetDevice(x->device);
    if (e == hipSuccess) e = hipMalloc(&x->scratch, sizeof(int32_t) * (mix::kScratchHead + (size_t)max_batch));
    for (int b = 0; b < x->nside() && e == hipSuccess; ++b) {
        e = hipStreamCreateWithFlags(&x->side[b], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x->ev_join[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&x->ev_fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (x->scratch) (void)hipFree(x->scratch);
        for (int b = 0; b < qldpc_mixed_s::kBranches; ++b) {
            if (x->side[b]) (void)hipStreamDestroy(x->side[b]);
            if (x->ev_join[b]) (void)hipEventDestroy(x->ev_join[b]);
        }
        if (x->ev_fork) (void)hipEventDestroy(x->ev_fork);
        delete x;
        return set_error(QLDPC_ERR_OUT_OF_MEMORY, "mixed_create: scratch, stream or event allocation");
    }
    *out = x;
    return QLDPC_OK;
}

qldpc_status qldpc_mixed_destroy(qldpc_mixed x) {
    if (!x) return QLDPC_OK;
    for (auto &kv : x->graphs) (void)hipGraphExecDestroy(kv.second);
    for (int b = 0; b < qldpc_mixed_s::kBranches; ++b)
        if (x->side[b]) (void)hipStreamSynchronize(x->side[b]);
    if (x->scratch) (void)hipFree(x->scratch);
    for (int b = 0; b < qldpc_mixed_s::kBranches; ++b) {
        if (x->side[b]) (void)hipStreamDestroy(x->side[b]);
        if (x->ev_join[b]) (void)hipEventDestroy(x->ev_join[b]);
    }
    if (x->ev_fork) (void)hipEventDestroy(x->ev_fork);
    delete x;
    return QLDPC_OK;
}

qldpc_status qldpc_mixed_decode(qldpc_mixed x, int32_t batch, const int32_t *shot_code, const int64_t *syn_off,
                                const int64_t *err_off, const uint32_t *syn, const float *prior, uint32_t *err,
                                uint8_t *conv, uint8_t *iters, void *stream) {
    if (!x) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_decode: null plan");
    if (batch < 0 || batch > x->max_batch) return set_error(QLDPC_ERR_INVALID_ARG, "mixed_decode: batch out of range");
    if (batch == 0) return QLDPC_OK;
    if (!shot_code || !syn_off || !err_off || !syn || !prior || !err || !conv)
        return set_error(QLDPC_ERR_INVALID_ARG, "mixed_decode: null buffer");
    hipStream_t st = (hipStream_t)stream;
    if (!x->use_graph) return enqueue(x, batch, shot_code, syn_off, err_off, syn, prior, err, conv, iters, st, x->waves);
    std::lock_guard<std::mutex> g(x->mu);
    auto key = std::make_tuple(batch, (const void *)shot_code, (const void *)syn_off, (const void *)err_off,
                               (const void *)syn, (const void *)prior, (const void *)err, (const void *)conv,
                               (const void *)iters, (const void *)nullptr, (void *)st, x->waves);
    auto it = x->graphs.find(key);
    hipGraphExec_t ex = nullptr;
    if (it == x->graphs.end()) {
        if (x->graphs.size() >= 16) {
            for (auto &kv : x->graphs) (void)hipGraphExecDestroy(kv.second);
            x->graphs.clear();
        }
        // capture on a private stream so the caller's stream is never in capture mode
        hipStream_t cs = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_error(e, "mixed_decode: capture stream");
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return hip_error(e, "mixed_decode: begin capture");
        }
        qldpc_status s2 = enqueue(x, batch, shot_code, syn_off, err_off, syn, prior, err, conv, iters, cs, x->waves);
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(cs, &gr);
        (void)hipStreamDestroy(cs);
        if (s2 != QLDPC_OK) {
            if (gr) (void)hipGraphDestroy(gr);
            return s2;
        }
        if (e != hipSuccess) return hip_error(e, "mixed_decode: end capture");
        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_error(e, "mixed_decode: instantiate");
        x->graphs[key] = ex;
    } else {
        ex = it->second;
    }
    hipError_t e = hipGraphLaunch(ex, st);
    if (e != hipSuccess) return hip_error(e, "mixed_decode: graph launch");
    return QLDPC_OK;
}

qldpc_status qldpc_mixed_set_grid(qldpc_mixed x, int32_t reg_waves, int32_t block_workgroups) {
    if (!x || reg_waves < 0 || block_workgroups < 0)
        return set_error(QLDPC_ERR_INVALID_ARG, "mixed_set_grid: bad arguments");
    std::lock_guard<std::mutex> g(x->mu);
    if (reg_waves > 0) x->waves = reg_waves;
    if (block_workgroups > 0) x->waves128 = block_workgroups;
    for (auto &kv : x->graphs) (void)hipGraphExecDestroy(kv.second);
    x->graphs.clear();
    return QLDPC_OK;
}

qldpc_status qldpc_mixed_autotune(qldpc_mixed x, int32_t batch, const int32_t *shot_code, const int64_t *syn_off,
                                  const int64_t *err_off, const uint32_t *syn, const float *prior, uint32_t *err,
                                  uint8_t *conv, uint8_t *iters, void *stream, int32_t *best_waves) {
    if (!x || batch <= 0 || batch > x->max_batch || !best_waves)
        return set_error(QLDPC_ERR_INVALID_ARG, "mixed_autotune: bad arguments");
    if (!shot_code || !syn_off || !err_off || !syn || !prior || !err || !conv)
        return set_error(QLDPC_ERR_INVALID_ARG, "mixed_autotune: null buffer");
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, x->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(QLDPC_ERR_DEVICE, "mixed_autotune: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(QLDPC_ERR_DEVICE, "mixed_autotune: event");
    }
    float best = 1e30f;
    int bw = x->waves;
    qldpc_status rc = QLDPC_OK;
    for (int mult : {6, 12, 24, 48}) {
        const int w = mult * cus;
        rc = enqueue(x, batch, shot_code, syn_off, err_off, syn, prior, err, conv, iters, st, w);
        if (rc != QLDPC_OK) break;
        hipError_t he = hipEventRecord(e0, st);
        for (int r = 0; r < 3 && rc == QLDPC_OK && he == hipSuccess; ++r)
            rc = enqueue(x, batch, shot_code, syn_off, err_off, syn, prior, err, conv, iters, st, w);
        if (he == hipSuccess) he = hipEventRecord(e1, st);
        if (rc != QLDPC_OK) break;
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = hip_error(he, "mixed_autotune: timing");
            break;
        }
        if (ms < best) {
            best = ms;
            bw = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != QLDPC_OK) return rc;
    std::lock_guard<std::mutex> g(x->mu);
    x->waves = bw;
    *best_waves = bw;
    return QLDPC_OK;
}

}  // extern "C"
