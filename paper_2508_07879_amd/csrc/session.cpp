// Latency sessions: host syndromes in, host decisions out, timed end to end
// as the paper's latency figure counts it (host-to-device copy, decode,
// device-to-host copy; Section 3).
//
// QLDPC_IO_COPY: inputs are copied into pinned staging, then a hipGraph
// captured once per batch size replays copy-in -> decode -> copy-out on the
// session's stream.  QLDPC_IO_MAPPED: the decoder reads the pinned staging
// and writes its results there directly (the GPU reaches host memory over
// the bus), so a request is one kernel launch.  QLDPC_IO_RESIDENT: as MAPPED,
// but the decoder stays resident between requests and is woken through a
// doorbell page in host memory, so a request is a few host stores and a spin
// on the answer: no launch, no stream synchronisation.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstring>
#include <map>
#include <new>
#include <thread>

#include "internal.h"

using namespace qldpc;

struct qldpc_session_s {
    qldpc_code code = nullptr;
    qldpc_decode_params params{};
    int32_t max_batch = 0;          // shots
    int32_t unit = 1;               // shots per request item: 2 for a CSS pair session
    int32_t io_mode = 0;
    int32_t syn_words = 0, err_words = 0;
    size_t prior_bytes_per_shot = 0;
    hipStream_t stream = nullptr;
    // device buffers (COPY mode)
    uint32_t *d_syn = nullptr;
    void *d_prior = nullptr;
    uint32_t *d_err = nullptr;
    uint8_t *d_conv = nullptr, *d_iters = nullptr;
    // pinned host staging
    uint32_t *h_syn = nullptr;
    void *h_prior = nullptr;
    uint32_t *h_err = nullptr;
    uint8_t *h_conv = nullptr, *h_iters = nullptr;
    // device-side addresses of the staging buffers (MAPPED mode)
    uint32_t *m_syn = nullptr;
    void *m_prior = nullptr;
    uint32_t *m_err = nullptr;
    uint8_t *m_conv = nullptr, *m_iters = nullptr;
    std::map<int32_t, hipGraphExec_t> graphs;
    // RESIDENT mode
    ResidentRing *ring = nullptr;     // doorbell page, host address
    uint64_t *d_cmd = nullptr;        // device mailbox of the resident grid
    hipEvent_t ev_exit = nullptr;     // recorded after each launch of the grid
    LaunchKey rkey{};
    ResidentArgs rargs{};
    uint64_t seq = 0;                 // sequence number of the last request
    bool running = false;             // a grid was launched and not seen to exit
    std::chrono::steady_clock::time_point last_answer{};
};

namespace {

// A resident grid leaves after this long without a request; the next request
// then relaunches it.
constexpr double kResidentIdleMs = 200.0;
// A request that has no answer after this long fails with QLDPC_ERR_DEVICE.
constexpr double kResidentTimeoutMs = 10000.0;

// Asks a resident grid to leave and waits (bounded) until it has; false if
// it is still running after kResidentTimeoutMs.
bool resident_stop(qldpc_session s) {
    if (!s->ring) return true;
    __atomic_store_n(&s->ring->stop, 1, __ATOMIC_SEQ_CST);
    const auto t0 = std::chrono::steady_clock::now();
    while (s->stream && hipStreamQuery(s->stream) == hipErrorNotReady) {
        if (std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() >
            kResidentTimeoutMs)
            return false;
        std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    s->running = false;
    return true;
}

void release(qldpc_session s) {
    if (s->ring) (void)hipHostFree(s->ring);
    if (s->ev_exit) (void)hipEventDestroy(s->ev_exit);
    if (s->d_cmd) (void)hipFree(s->d_cmd);
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    if (s->d_syn) (void)hipFree(s->d_syn);
    if (s->d_prior) (void)hipFree(s->d_prior);
    if (s->d_err) (void)hipFree(s->d_err);
    if (s->d_conv) (void)hipFree(s->d_conv);
    if (s->d_iters) (void)hipFree(s->d_iters);
    if (s->h_syn) (void)hipHostFree(s->h_syn);
    if (s->h_prior) (void)hipHostFree(s->h_prior);
    if (s->h_err) (void)hipHostFree(s->h_err);
    if (s->h_conv) (void)hipHostFree(s->h_conv);
    if (s->h_iters) (void)hipHostFree(s->h_iters);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

// Enqueues one decode of `batch` shots from the staging buffers.
qldpc_status enqueue(qldpc_session s, int32_t batch) {
    LaunchKey k{};
    DecodeArgs a{};
    qldpc_status st = prepare_decode(s->code, &s->params, batch, &k, &a);
    if (st != QLDPC_OK) return st;
    if (s->io_mode == QLDPC_IO_MAPPED) {
        a.syn = s->m_syn;
        a.prior = s->m_prior;
        a.err = s->m_err;
        a.conv = s->m_conv;
        a.iters = s->m_iters;
    } else {
        a.syn = s->d_syn;
        a.prior = s->d_prior;
        a.err = s->d_err;
        a.conv = s->d_conv;
        a.iters = s->d_iters;
    }
    a.post = nullptr;
    k.post = 0;
    hipError_t e = launch_code_decode(s->code, k, a, s->stream);
    if (e == hipErrorNotSupported) return set_error(QLDPC_ERR_UNSUPPORTED, "session: no kernel for these parameters");
    if (e != hipSuccess) return hip_error(e, "session: launch");
    return QLDPC_OK;
}

qldpc_status graph_for(qldpc_session s, int32_t batch, hipGraphExec_t *out) {
    auto it = s->graphs.find(batch);
    if (it != s->graphs.end()) {
        *out = it->second;
        return QLDPC_OK;
    }
    hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_error(e, "session: begin capture");
    qldpc_status st = QLDPC_OK;
    const size_t sb = (size_t)batch * s->syn_words * 4, pb = (size_t)batch * s->prior_bytes_per_shot;
    const size_t eb = (size_t)batch * s->err_words * 4;
    hipError_t ce = hipMemcpyAsync(s->d_syn, s->h_syn, sb, hipMemcpyHostToDevice, s->stream);
    if (ce == hipSuccess) ce = hipMemcpyAsync(s->d_prior, s->h_prior, pb, hipMemcpyHostToDevice, s->stream);
    if (ce == hipSuccess) st = enqueue(s, batch);
    if (ce == hipSuccess && st == QLDPC_OK) ce = hipMemcpyAsync(s->h_err, s->d_err, eb, hipMemcpyDeviceToHost, s->stream);
    if (ce == hipSuccess && st == QLDPC_OK)
        ce = hipMemcpyAsync(s->h_conv, s->d_conv, (size_t)batch, hipMemcpyDeviceToHost, s->stream);
    if (ce == hipSuccess && st == QLDPC_OK)
        ce = hipMemcpyAsync(s->h_iters, s->d_iters, (size_t)batch, hipMemcpyDeviceToHost, s->stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(s->stream, &g);   // always end the capture, whatever failed inside it
    if (st != QLDPC_OK || ce != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return st != QLDPC_OK ? st : hip_error(ce, "session: capture copy");
    }
    if (e != hipSuccess) return hip_error(e, "session: end capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_error(e, "session: instantiate");
    s->graphs[batch] = ex;
    *out = ex;
    return QLDPC_OK;
}

// Launches the resident grid, which then serves every request numbered after
// `served`.
qldpc_status resident_start(qldpc_session s, uint64_t served) {
    ResidentArgs r = s->rargs;
    r.start_seq = served;
    hipError_t e = launch_resident_decode(s->rkey, r, s->max_batch, s->stream);
    if (e == hipErrorNotSupported) return set_error(QLDPC_ERR_UNSUPPORTED, "session: no resident kernel for these parameters");
    if (e != hipSuccess) return hip_error(e, "session: resident launch");
    e = hipEventRecord(s->ev_exit, s->stream);
    if (e != hipSuccess) return hip_error(e, "session: record");
    s->running = true;
    return QLDPC_OK;
}

// Whether the last launched grid is still on the GPU.
qldpc_status resident_alive(qldpc_session s, bool *alive) {
    *alive = false;
    if (!s->running) return QLDPC_OK;
    const hipError_t q = hipEventQuery(s->ev_exit);
    if (q == hipErrorNotReady) {
        *alive = true;
        return QLDPC_OK;
    }
    s->running = false;
    if (q != hipSuccess) return hip_error(q, "session: resident grid");
    return QLDPC_OK;
}

qldpc_status run_resident(qldpc_session s, int32_t batch) {
    using clk = std::chrono::steady_clock;
    // A grid idle for about kResidentIdleMs may have left; ask the runtime only then.
    const double since = std::chrono::duration<double, std::milli>(clk::now() - s->last_answer).count();
    if (!s->running || since > 0.5 * kResidentIdleMs) {
        bool alive = false;
        qldpc_status st = resident_alive(s, &alive);
        if (st == QLDPC_OK && !alive) st = resident_start(s, s->seq);
        if (st != QLDPC_OK) return st;
    }
    const uint64_t seq = s->seq + 1;
    std::atomic_thread_fence(std::memory_order_seq_cst);   // staged inputs before the doorbell
    __atomic_store_n(&s->ring->batch, batch, __ATOMIC_RELAXED);
    __atomic_store_n(&s->ring->req_seq, seq, __ATOMIC_RELEASE);
    s->seq = seq;
    const auto t0 = clk::now();
    for (uint32_t spin = 1;; ++spin) {
        int32_t w = 0;
        while (w < batch && __atomic_load_n(&s->ring->done_seq[w], __ATOMIC_ACQUIRE) == seq) ++w;
        if (w == batch) break;
        if ((spin & 4095) == 0) {
            // the grid may have timed out just before the doorbell rang
            bool alive = false;
            qldpc_status st = resident_alive(s, &alive);
            if (st == QLDPC_OK && !alive) st = resident_start(s, seq - 1);
            if (st != QLDPC_OK) return st;
            if (std::chrono::duration<double, std::milli>(clk::now() - t0).count() > kResidentTimeoutMs)
                return set_error(QLDPC_ERR_DEVICE, "session: the resident decoder did not answer");
        }
        __builtin_ia32_pause();
    }
    s->last_answer = clk::now();
    return QLDPC_OK;
}

// Decode from the staging buffers, synchronously.
qldpc_status run_staged(qldpc_session s, int32_t batch) {
    hipError_t e;
    if (s->io_mode == QLDPC_IO_RESIDENT) return run_resident(s, batch);
    if (s->io_mode == QLDPC_IO_MAPPED) {
        qldpc_status st = enqueue(s, batch);
        if (st != QLDPC_OK) return st;
    } else {
        hipGraphExec_t g = nullptr;
        qldpc_status st = graph_for(s, batch, &g);
        if (st != QLDPC_OK) return st;
        e = hipGraphLaunch(g, s->stream);
        if (e != hipSuccess) return hip_error(e, "session: graph launch");
    }
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_error(e, "session: synchronize");
    return QLDPC_OK;
}

// A session over `max_batch` shots; code_x (CSS pairs, resident only): the
// H_X side, decoding the odd shots.
qldpc_status session_create_impl(qldpc_code code, qldpc_code code_x, const qldpc_decode_params *params,
                                 int32_t max_batch, int32_t io_mode, qldpc_session *out) {
    if (!code || !params || !out) return set_error(QLDPC_ERR_INVALID_ARG, "session_create: null argument");
    if (max_batch <= 0) return set_error(QLDPC_ERR_INVALID_ARG, "session_create: max_batch must be positive");
    if (io_mode != QLDPC_IO_COPY && io_mode != QLDPC_IO_MAPPED && io_mode != QLDPC_IO_RESIDENT)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_create: bad io mode");
    const bool resident = io_mode == QLDPC_IO_RESIDENT;
    if (resident && max_batch > kMaxResident)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_create: a resident session takes at most 64 shots");
    qldpc_decode_params prm = *params;
    if (resident) prm.layout = QLDPC_LAYOUT_BLOCK;   // the resident grid is workgroup-per-shot
    LaunchKey k{};
    DecodeArgs a{};
    qldpc_status st = prepare_decode(code, &prm, max_batch, &k, &a);   // validates params
    if (st != QLDPC_OK) return st;
    if (k.layout == QLDPC_LAYOUT_HBM)
        return set_error(QLDPC_ERR_UNSUPPORTED, "session_create: sessions keep messages on chip (no HBM layout)");
    params = &prm;
    auto *s = new (std::nothrow) qldpc_session_s();
    if (!s) return set_error(QLDPC_ERR_OUT_OF_MEMORY, "session_create: host allocation");
    s->code = code;
    s->params = *params;
    s->max_batch = max_batch;
    s->unit = code_x ? 2 : 1;
    s->io_mode = io_mode;
    s->syn_words = (code->m + 31) / 32;
    s->err_words = (code->n + 31) / 32;
    const size_t vbytes = params->fmt == QLDPC_F32 ? 4 : params->fmt == QLDPC_I16Q8 ? 2 : 1;
    s->prior_bytes_per_shot = params->prior_mode == QLDPC_PRIOR_PER_BIT ? vbytes * code->n : vbytes;
    const size_t B = (size_t)max_batch;
    // MAPPED: fine-grained (coherent) pinned memory the kernel reads and writes
    // over the bus; COPY: ordinary pinned staging for the copy engines.
    const bool mapped = io_mode != QLDPC_IO_COPY;
    const unsigned fl = mapped ? (hipHostMallocMapped | hipHostMallocCoherent) : hipHostMallocDefault;
    hipError_t e = hipSetDevice(code->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_syn, B * s->syn_words * 4, fl);
    if (e == hipSuccess) e = hipHostMalloc(&s->h_prior, B * s->prior_bytes_per_shot, fl);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_err, B * s->err_words * 4, fl);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_conv, B, fl);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_iters, B, fl);
    if (e == hipSuccess && mapped) {
        e = hipHostGetDevicePointer((void **)&s->m_syn, s->h_syn, 0);
        if (e == hipSuccess) e = hipHostGetDevicePointer(&s->m_prior, s->h_prior, 0);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->m_err, s->h_err, 0);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->m_conv, s->h_conv, 0);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->m_iters, s->h_iters, 0);
    }
    if (e == hipSuccess && io_mode == QLDPC_IO_COPY) {
        e = hipMalloc((void **)&s->d_syn, B * s->syn_words * 4);
        if (e == hipSuccess) e = hipMalloc(&s->d_prior, B * s->prior_bytes_per_shot);
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_err, B * s->err_words * 4);
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_conv, B);
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_iters, B);
    }
    ResidentRing *m_ring = nullptr;
    int clock_khz = 0;
    if (e == hipSuccess && resident) {
        e = hipHostMalloc((void **)&s->ring, sizeof(ResidentRing), hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) {
            std::memset(s->ring, 0, sizeof(ResidentRing));
            e = hipHostGetDevicePointer((void **)&m_ring, s->ring, 0);
        }
        if (e == hipSuccess) e = hipMalloc((void **)&s->d_cmd, 2 * sizeof(uint64_t));
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_exit, hipEventDisableTiming);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, code->device);
    }
    if (e != hipSuccess) {
        release(s);
        return set_error(QLDPC_ERR_OUT_OF_MEMORY, std::string("session_create: ") + hipGetErrorString(e));
    }
    if (resident) {
        s->rkey = k;
        s->rkey.post = 0;
        if (code_x) s->rkey.which = 2;
        s->rargs.a = a;
        s->rargs.code_x = code_x ? code_x->dev : nullptr;
        s->rargs.a.syn = s->m_syn;
        s->rargs.a.prior = s->m_prior;
        s->rargs.a.err = s->m_err;
        s->rargs.a.conv = s->m_conv;
        s->rargs.a.iters = s->m_iters;
        s->rargs.a.post = nullptr;
        s->rargs.ring = m_ring;
        s->rargs.cmd = s->d_cmd;
        s->rargs.idle_ticks = (uint64_t)(kResidentIdleMs * (clock_khz > 0 ? clock_khz : 100000));
        st = resident_start(s, 0);
        if (st != QLDPC_OK) {
            if (resident_stop(s)) release(s);
            return st;
        }
        s->last_answer = std::chrono::steady_clock::now();
    }
    *out = s;
    return QLDPC_OK;
}

}  // namespace

extern "C" {

qldpc_status qldpc_session_create(qldpc_code code, const qldpc_decode_params *params, int32_t max_batch,
                                  int32_t io_mode, qldpc_session *out) {
    return session_create_impl(code, nullptr, params, max_batch, io_mode, out);
}

qldpc_status qldpc_session_create_css(qldpc_code hz_side, qldpc_code hx_side, const qldpc_decode_params *params,
                                      int32_t max_pairs, qldpc_session *out) {
    if (!hz_side || !hx_side || !params || !out) return set_error(QLDPC_ERR_INVALID_ARG, "session_create_css: null argument");
    if (max_pairs <= 0 || 2 * max_pairs > kMaxResident)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_create_css: max_pairs must be in [1, 32]");
    if (hz_side->which != 0 || hx_side->which != 1)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_create_css: needs an H_Z-pattern and an H_X-pattern code");
    if (hz_side->L != hx_side->L || hz_side->m != hx_side->m || hz_side->n != hx_side->n ||
        hz_side->device != hx_side->device)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_create_css: the two sides differ in lift, size or device");
    if (params->fmt != QLDPC_F32 && params->fmt != QLDPC_I8Q4)
        return set_error(QLDPC_ERR_UNSUPPORTED, "session_create_css: FP32 or int8 messages");
    return session_create_impl(hz_side, hx_side, params, 2 * max_pairs, QLDPC_IO_RESIDENT, out);
}

qldpc_status qldpc_session_destroy(qldpc_session s) {
    if (!s) return QLDPC_OK;
    if (!resident_stop(s))   // leave the buffers to a grid that still runs rather than free them under it
        return set_error(QLDPC_ERR_DEVICE, "session_destroy: the resident decoder did not exit; session leaked");
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    release(s);
    return QLDPC_OK;
}

qldpc_status qldpc_session_decode(qldpc_session s, int32_t batch, const uint32_t *host_syn,
                                  const void *host_prior, uint32_t *host_err, uint8_t *host_conv,
                                  uint8_t *host_iters) {
    if (!s) return set_error(QLDPC_ERR_INVALID_ARG, "session_decode: null session");
    if (batch < 0 || batch > s->max_batch / s->unit)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_decode: batch out of range");
    if (batch == 0) return QLDPC_OK;
    batch *= s->unit;   // shots
    if (!host_syn || !host_prior) return set_error(QLDPC_ERR_INVALID_ARG, "session_decode: null input");
    std::memcpy(s->h_syn, host_syn, (size_t)batch * s->syn_words * 4);
    std::memcpy(s->h_prior, host_prior, (size_t)batch * s->prior_bytes_per_shot);
    qldpc_status st = run_staged(s, batch);
    if (st != QLDPC_OK) return st;
    if (host_err) std::memcpy(host_err, s->h_err, (size_t)batch * s->err_words * 4);
    if (host_conv) std::memcpy(host_conv, s->h_conv, (size_t)batch);
    if (host_iters) std::memcpy(host_iters, s->h_iters, (size_t)batch);
    return QLDPC_OK;
}

qldpc_status qldpc_session_latency(qldpc_session s, int32_t nreq, int32_t batch, int32_t pool,
                                   const uint32_t *host_syn, const void *host_prior, double *lat_us) {
    if (!s || !host_syn || !host_prior || !lat_us) return set_error(QLDPC_ERR_INVALID_ARG, "session_latency: null argument");
    if (nreq < 0 || batch <= 0 || batch > s->max_batch / s->unit || pool < batch)
        return set_error(QLDPC_ERR_INVALID_ARG, "session_latency: bad sizes");
    const int64_t u = s->unit;   // shots per item
    std::vector<uint32_t> err((size_t)(batch * u) * s->err_words);
    std::vector<uint8_t> conv(batch * u), it(batch * u);
    const char *pr = static_cast<const char *>(host_prior);
    for (int32_t i = 0; i < nreq; ++i) {
        int64_t start = ((int64_t)i * batch) % pool;
        if (start + batch > pool) start = 0;
        const auto t0 = std::chrono::steady_clock::now();
        qldpc_status st = qldpc_session_decode(s, batch, host_syn + start * u * s->syn_words,
                                               pr + start * u * s->prior_bytes_per_shot, err.data(), conv.data(),
                                               it.data());
        const auto t1 = std::chrono::steady_clock::now();
        if (st != QLDPC_OK) return st;
        lat_us[i] = std::chrono::duration<double, std::micro>(t1 - t0).count();
    }
    return QLDPC_OK;
}

}  // extern "C"
