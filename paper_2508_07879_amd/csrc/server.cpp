// Continuous-batching decode server (the paper's proposal of several
// asynchronous decoders overlapping transfers and kernels, Table 1 and
// Section 3, realised as a request loop).
//
// Requests (1..max_batch_shots syndromes of one code, plain or neural
// min-sum) enter a bounded queue.  A scheduler thread owns a fixed set of
// slots -- device buffers, pinned staging, a stream and a mixed-code plan
// each -- whose number is set by the HBM budget.  Whenever a slot is free it
// admits queued requests (FIFO, up to the slot's shot capacity) as one
// micro-batch: copy-in, one mixed-code persistent decode for the plain
// min-sum shots, one neural decode per code for the neural shots, copy-out,
// event.  Micro-batches on different slots overlap on the device.  Finished
// slots scatter their results into the requests' host buffers and post
// completions.  Every shot's result is that of decoding it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <random>
#include <thread>
#include <vector>

#include "internal.h"

using namespace qldpc;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t id;
    int32_t code, decoder, nshots;
    const uint32_t *syn;
    const float *prior;
    uint32_t *err;
    uint8_t *conv, *iters;
    int64_t t_submit;
    // placement inside the slot's micro-batch
    int32_t first_shot;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    qldpc_mixed plan = nullptr;
    int32_t *d_cid = nullptr, *h_cid = nullptr;
    int64_t *d_soff = nullptr, *h_soff = nullptr, *d_eoff = nullptr, *h_eoff = nullptr;
    uint32_t *d_syn = nullptr, *h_syn = nullptr, *d_err = nullptr, *h_err = nullptr;
    float *d_prior = nullptr, *h_prior = nullptr;
    uint8_t *d_conv = nullptr, *h_conv = nullptr, *d_iters = nullptr, *h_iters = nullptr, *d_used = nullptr;
    std::vector<Request> reqs;
    bool busy = false;
    int32_t shots = 0;
    int64_t syn_words = 0, err_words = 0;
};

}  // namespace

struct qldpc_server_s {
    qldpc_server_config cfg{};
    std::vector<qldpc_code> codes;
    std::vector<const float *> weights;
    int32_t max_sw = 0, max_ew = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending;
    std::vector<qldpc_completion> completions;
    std::atomic<bool> stop{false};
    std::atomic<int64_t> inflight_shots{0};
    qldpc_status worker_status = QLDPC_OK;
    std::string worker_error;
    std::thread worker;
    size_t slot_bytes = 0;
    // Failure injection for tests of the error path: the launch of this
    // micro-batch (1-based count) fails before anything is enqueued
    // (environment variable QLDPC_TEST_FAIL_LAUNCH at create time; 0 = never).
    int64_t fail_launch_at = 0;
    int64_t launches = 0;
};

namespace {

template <class T>
hipError_t dev_alloc(T **p, size_t n) { return hipMalloc((void **)p, n * sizeof(T)); }
template <class T>
hipError_t host_alloc(T **p, size_t n) { return hipHostMalloc((void **)p, n * sizeof(T), hipHostMallocDefault); }

void free_slot(Slot &s) {
    if (s.plan) qldpc_mixed_destroy(s.plan);
    for (void *d : {(void *)s.d_cid, (void *)s.d_soff, (void *)s.d_eoff, (void *)s.d_syn, (void *)s.d_err,
                    (void *)s.d_prior, (void *)s.d_conv, (void *)s.d_iters, (void *)s.d_used})
        if (d) (void)hipFree(d);
    for (void *h : {(void *)s.h_cid, (void *)s.h_soff, (void *)s.h_eoff, (void *)s.h_syn, (void *)s.h_err,
                    (void *)s.h_prior, (void *)s.h_conv, (void *)s.h_iters})
        if (h) (void)hipHostFree(h);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot{};
}

// Device bytes one slot holds for `shots` shots.
size_t slot_device_bytes(int64_t shots, int32_t sw, int32_t ew) {
    return (size_t)shots * (4 + 8 + 8 + 4 * (size_t)sw + 4 * (size_t)ew + 4 + 1 + 1 + 1) + 4 * ((size_t)shots + 17);
}

// Packs the slot's requests into its staging and launches the micro-batch.
qldpc_status launch_slot(qldpc_server srv, Slot &s) {
    if (++srv->launches == srv->fail_launch_at)
        return set_error(QLDPC_ERR_DEVICE, "server: injected launch failure");
    const int32_t nc = (int32_t)srv->codes.size();
    // plain min-sum shots first (ragged, any code), then neural shots per code
    int32_t shot = 0;
    int64_t sw_at = 0, ew_at = 0;
    std::vector<int32_t> nms_first(nc, -1), nms_count(nc, 0);
    std::vector<int64_t> nms_sw(nc, 0), nms_ew(nc, 0);
    auto place = [&](Request &r) {
        const qldpc_code c = srv->codes[r.code];
        const int32_t sw = (c->m + 31) / 32, ew = (c->n + 31) / 32;
        r.first_shot = shot;
        for (int32_t i = 0; i < r.nshots; ++i) {
            s.h_cid[shot] = r.code;
            s.h_soff[shot] = sw_at;
            s.h_eoff[shot] = ew_at;
            std::memcpy(s.h_syn + sw_at, r.syn + (size_t)i * sw, sizeof(uint32_t) * sw);
            s.h_prior[shot] = r.prior[i];
            sw_at += sw;
            ew_at += ew;
            ++shot;
        }
    };
    for (Request &r : s.reqs)
        if (r.decoder == 0) place(r);
    const int32_t n_plain = shot;
    for (int32_t c = 0; c < nc; ++c) {
        for (Request &r : s.reqs)
            if (r.decoder == 1 && r.code == c) {
                if (nms_first[c] < 0) {
                    nms_first[c] = shot;
                    nms_sw[c] = sw_at;
                    nms_ew[c] = ew_at;
                }
                nms_count[c] += r.nshots;
                place(r);
            }
    }
    s.shots = shot;
    s.syn_words = sw_at;
    s.err_words = ew_at;
    hipStream_t st = s.stream;
    hipError_t e = hipSuccess;
    if (n_plain > 0) {
        e = hipMemcpyAsync(s.d_cid, s.h_cid, sizeof(int32_t) * n_plain, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_soff, s.h_soff, sizeof(int64_t) * n_plain, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_eoff, s.h_eoff, sizeof(int64_t) * n_plain, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(s.d_syn, s.h_syn, sizeof(uint32_t) * sw_at, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s.d_prior, s.h_prior, sizeof(float) * shot, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_error(e, "server: copy-in");
    qldpc_status rc = QLDPC_OK;
    if (n_plain > 0)
        rc = qldpc_mixed_decode(s.plan, n_plain, s.d_cid, s.d_soff, s.d_eoff, s.d_syn, s.d_prior, s.d_err, s.d_conv,
                                s.d_iters, st);
    for (int32_t c = 0; c < nc && rc == QLDPC_OK; ++c) {
        if (nms_count[c] == 0) continue;
        const int32_t f = nms_first[c];
        rc = qldpc_nbp_decode(srv->codes[c], nms_count[c], srv->cfg.nms_T, srv->weights[c], &srv->cfg.params,
                              s.d_syn + nms_sw[c], s.d_prior + f, s.d_err + nms_ew[c], s.d_conv + f,
                              s.d_iters + f, s.d_used + f, st);
    }
    if (rc != QLDPC_OK) return rc;
    e = hipMemcpyAsync(s.h_err, s.d_err, sizeof(uint32_t) * ew_at, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_conv, s.d_conv, shot, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_iters, s.d_iters, shot, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(s.done, st);
    if (e != hipSuccess) return hip_error(e, "server: copy-out");
    return QLDPC_OK;
}

qldpc_completion completion_of(const Request &r, qldpc_status status, int64_t t) {
    qldpc_completion q{};
    q.req_id = r.id;
    q.code_id = r.code;
    q.decoder = r.decoder;
    q.nshots = r.nshots;
    q.status = status;
    q.t_submit_ns = r.t_submit;
    q.t_done_ns = t;
    return q;
}

// Retires a slot: on success scatters its results into the requests' host
// buffers; on failure leaves those buffers untouched.  Either way every
// request of the slot gets one completion carrying `status`.
void finish_slot(qldpc_server srv, Slot &s, qldpc_status status) {
    const int64_t t = now_ns();
    std::vector<qldpc_completion> done;
    done.reserve(s.reqs.size());
    for (const Request &r : s.reqs) {
        if (status == QLDPC_OK) {
            const qldpc_code c = srv->codes[r.code];
            const int32_t ew = (c->n + 31) / 32;
            for (int32_t i = 0; i < r.nshots; ++i) {
                const int32_t sh = r.first_shot + i;
                if (r.err) std::memcpy(r.err + (size_t)i * ew, s.h_err + s.h_eoff[sh], sizeof(uint32_t) * ew);
                if (r.conv) r.conv[i] = s.h_conv[sh];
                if (r.iters) r.iters[i] = s.h_iters[sh];
            }
        }
        done.push_back(completion_of(r, status, t));
    }
    srv->inflight_shots -= s.shots;
    s.reqs.clear();
    s.shots = 0;
    s.busy = false;
    std::lock_guard<std::mutex> g(srv->mu);
    srv->completions.insert(srv->completions.end(), done.begin(), done.end());
}

// Records the first failure; the server then stops admitting, and the
// requests still queued complete with that status.
void fail_server(qldpc_server srv, qldpc_status st, const std::string &msg) {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->worker_status == QLDPC_OK) {
        srv->worker_status = st;
        srv->worker_error = msg;
    }
    srv->stop = true;
    const int64_t t = now_ns();
    for (const Request &r : srv->pending) srv->completions.push_back(completion_of(r, srv->worker_status, t));
    srv->pending.clear();
}

void worker_loop(qldpc_server srv) {
    (void)hipSetDevice(srv->codes[0]->device);
    const int32_t cap = srv->cfg.max_batch_shots;
    while (true) {
        bool progressed = false;
        // retire finished slots
        for (Slot &s : srv->slots) {
            if (!s.busy) continue;
            hipError_t q = hipEventQuery(s.done);
            if (q == hipSuccess) {
                finish_slot(srv, s, QLDPC_OK);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                fail_server(srv, QLDPC_ERR_DEVICE, std::string("server: ") + hipGetErrorString(q));
                (void)hipStreamSynchronize(s.stream);
                finish_slot(srv, s, QLDPC_ERR_DEVICE);
                progressed = true;
            }
        }
        // admit queued requests into free slots
        for (Slot &s : srv->slots) {
            if (srv->stop) break;
            if (s.busy) continue;
            {
                std::lock_guard<std::mutex> g(srv->mu);
                int32_t shots = 0;
                while (!srv->pending.empty() && shots + srv->pending.front().nshots <= cap) {
                    shots += srv->pending.front().nshots;
                    s.reqs.push_back(srv->pending.front());
                    srv->pending.pop_front();
                }
            }
            if (s.reqs.empty()) break;
            s.busy = true;
            int32_t n = 0;
            for (auto &r : s.reqs) n += r.nshots;
            srv->inflight_shots += n;
            qldpc_status rc = launch_slot(srv, s);
            if (rc != QLDPC_OK) {
                // the micro-batch may be partly enqueued: wait for what was,
                // then fail its requests without touching their buffers
                fail_server(srv, rc, qldpc_last_error());
                (void)hipStreamSynchronize(s.stream);
                finish_slot(srv, s, rc);
            }
            progressed = true;
        }
        bool any_busy = false;
        for (Slot &s : srv->slots) any_busy = any_busy || s.busy;
        if (srv->stop && !any_busy) break;
        if (srv->stop && any_busy) {
            // drain: every busy slot was launched completely (its event is
            // recorded); wait for its stream, then retire
            for (Slot &s : srv->slots)
                if (s.busy) {
                    const hipError_t q = hipStreamSynchronize(s.stream);
                    finish_slot(srv, s, q == hipSuccess ? QLDPC_OK : QLDPC_ERR_DEVICE);
                }
            break;
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(srv->mu);
            if (srv->pending.empty() && !any_busy)
                srv->cv.wait_for(lk, std::chrono::microseconds(200));
            else
                std::this_thread::yield();
        }
    }
}

}  // namespace

extern "C" {

qldpc_status qldpc_server_create(const qldpc_server_config *cfg, qldpc_server *out) {
    if (!cfg || !out || !cfg->codes || cfg->ncodes < 1 || cfg->ncodes > 8)
        return set_error(QLDPC_ERR_INVALID_ARG, "server_create: bad configuration");
    if (cfg->max_batch_shots < 1 || cfg->max_inflight < 1 || cfg->queue_capacity < 1)
        return set_error(QLDPC_ERR_INVALID_ARG, "server_create: sizes must be positive");
    if (cfg->nms_weights && (cfg->nms_T < 1 || cfg->nms_T > 255))
        return set_error(QLDPC_ERR_INVALID_ARG, "server_create: nms_T must be in [1, 255]");
    for (int c = 0; c < cfg->ncodes; ++c) {
        if (!cfg->codes[c]) return set_error(QLDPC_ERR_INVALID_ARG, "server_create: null code");
        const int L = cfg->codes[c]->L;
        if (cfg->nms_weights && cfg->nms_weights[c] && (cfg->codes[c]->which != 0 || (L != 32 && L != 64 && L != 128)))
            return set_error(QLDPC_ERR_UNSUPPORTED,
                             "server_create: neural weights for H_Z-pattern codes with L = 32, 64 or 128 only");
    }
    auto *srv = new (std::nothrow) qldpc_server_s();
    if (!srv) return set_error(QLDPC_ERR_OUT_OF_MEMORY, "server_create: host allocation");
    srv->cfg = *cfg;
    if (const char *f = std::getenv("QLDPC_TEST_FAIL_LAUNCH")) srv->fail_launch_at = std::atoll(f);
    srv->codes.assign(cfg->codes, cfg->codes + cfg->ncodes);
    srv->weights.assign(cfg->ncodes, nullptr);
    for (int c = 0; c < cfg->ncodes; ++c) {
        if (cfg->nms_weights) srv->weights[c] = cfg->nms_weights[c];
        srv->max_sw = std::max(srv->max_sw, (srv->codes[c]->m + 31) / 32);
        srv->max_ew = std::max(srv->max_ew, (srv->codes[c]->n + 31) / 32);
    }
    const int64_t B = cfg->max_batch_shots;
    srv->slot_bytes = slot_device_bytes(B, srv->max_sw, srv->max_ew);
    int32_t nslots = cfg->max_inflight;
    if (cfg->hbm_budget > 0) nslots = (int32_t)std::min<size_t>(nslots, cfg->hbm_budget / srv->slot_bytes);
    if (nslots < 1) {
        delete srv;
        return set_error(QLDPC_ERR_CAPACITY, "server_create: HBM budget below one slot");
    }
    hipError_t e = hipSetDevice(srv->codes[0]->device);
    srv->slots.resize(nslots);
    qldpc_status rc = QLDPC_OK;
    for (Slot &s : srv->slots) {
        const size_t sw = (size_t)B * srv->max_sw, ew = (size_t)B * srv->max_ew;
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = dev_alloc(&s.d_cid, B);
        if (e == hipSuccess) e = dev_alloc(&s.d_soff, B);
        if (e == hipSuccess) e = dev_alloc(&s.d_eoff, B);
        if (e == hipSuccess) e = dev_alloc(&s.d_syn, sw);
        if (e == hipSuccess) e = dev_alloc(&s.d_err, ew);
        if (e == hipSuccess) e = dev_alloc(&s.d_prior, B);
        if (e == hipSuccess) e = dev_alloc(&s.d_conv, B);
        if (e == hipSuccess) e = dev_alloc(&s.d_iters, B);
        if (e == hipSuccess) e = dev_alloc(&s.d_used, B);
        if (e == hipSuccess) e = host_alloc(&s.h_cid, B);
        if (e == hipSuccess) e = host_alloc(&s.h_soff, B);
        if (e == hipSuccess) e = host_alloc(&s.h_eoff, B);
        if (e == hipSuccess) e = host_alloc(&s.h_syn, sw);
        if (e == hipSuccess) e = host_alloc(&s.h_err, ew);
        if (e == hipSuccess) e = host_alloc(&s.h_prior, B);
        if (e == hipSuccess) e = host_alloc(&s.h_conv, B);
        if (e == hipSuccess) e = host_alloc(&s.h_iters, B);
        if (e != hipSuccess) break;
        rc = qldpc_mixed_create(cfg->codes, cfg->ncodes, &cfg->params, (int32_t)B, 0, &s.plan);
        if (rc != QLDPC_OK) break;
    }
    if (e != hipSuccess || rc != QLDPC_OK) {
        for (Slot &s : srv->slots) free_slot(s);
        delete srv;
        return e != hipSuccess ? set_error(QLDPC_ERR_OUT_OF_MEMORY, "server_create: slot allocation") : rc;
    }
    srv->worker = std::thread(worker_loop, srv);
    *out = srv;
    return QLDPC_OK;
}

qldpc_status qldpc_server_info(qldpc_server srv, int32_t *slots, size_t *slot_bytes, int32_t *pending,
                               int64_t *inflight_shots) {
    if (!srv) return set_error(QLDPC_ERR_INVALID_ARG, "server_info: null server");
    if (slots) *slots = (int32_t)srv->slots.size();
    if (slot_bytes) *slot_bytes = srv->slot_bytes;
    if (pending) {
        std::lock_guard<std::mutex> g(srv->mu);
        *pending = (int32_t)srv->pending.size();
    }
    if (inflight_shots) *inflight_shots = srv->inflight_shots.load();
    return QLDPC_OK;
}

qldpc_status qldpc_server_submit(qldpc_server srv, int32_t code_id, int32_t decoder, int32_t nshots,
                                 const uint32_t *host_syn, const float *host_prior, uint32_t *host_err,
                                 uint8_t *host_conv, uint8_t *host_iters, uint64_t req_id) {
    if (!srv) return set_error(QLDPC_ERR_INVALID_ARG, "server_submit: null server");
    if (code_id < 0 || code_id >= (int32_t)srv->codes.size())
        return set_error(QLDPC_ERR_INVALID_ARG, "server_submit: bad code id");
    if (decoder != 0 && decoder != 1) return set_error(QLDPC_ERR_INVALID_ARG, "server_submit: decoder must be 0 or 1");
    if (decoder == 1 && !srv->weights[code_id])
        return set_error(QLDPC_ERR_UNSUPPORTED, "server_submit: no neural weights for this code");
    if (nshots < 1 || nshots > srv->cfg.max_batch_shots)
        return set_error(QLDPC_ERR_INVALID_ARG, "server_submit: nshots out of range");
    if (!host_syn || !host_prior) return set_error(QLDPC_ERR_INVALID_ARG, "server_submit: null input");
    Request r{req_id, code_id, decoder, nshots, host_syn, host_prior, host_err, host_conv, host_iters, now_ns(), 0};
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (srv->worker_status != QLDPC_OK) return set_error(srv->worker_status, srv->worker_error);
        if ((int32_t)srv->pending.size() >= srv->cfg.queue_capacity)
            return set_error(QLDPC_ERR_CAPACITY, "server_submit: queue full");
        srv->pending.push_back(r);
    }
    srv->cv.notify_one();
    return QLDPC_OK;
}

qldpc_status qldpc_server_poll(qldpc_server srv, qldpc_completion *out, int32_t max, int32_t *n_out) {
    if (!srv || !n_out || (max > 0 && !out)) return set_error(QLDPC_ERR_INVALID_ARG, "server_poll: bad arguments");
    std::lock_guard<std::mutex> g(srv->mu);
    const int32_t n = std::min<int32_t>(max, (int32_t)srv->completions.size());
    std::copy(srv->completions.begin(), srv->completions.begin() + n, out);
    srv->completions.erase(srv->completions.begin(), srv->completions.begin() + n);
    *n_out = n;
    if (srv->worker_status != QLDPC_OK) return set_error(srv->worker_status, srv->worker_error);
    return n > 0 ? QLDPC_OK : QLDPC_ERR_NOT_READY;
}

qldpc_status qldpc_server_destroy(qldpc_server srv) {
    if (!srv) return QLDPC_OK;
    srv->stop = true;
    srv->cv.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (Slot &s : srv->slots) free_slot(s);
    delete srv;
    return QLDPC_OK;
}

// Open-loop Poisson load: requests arrive at exponential intervals (mean
// request size / rate), their latency runs from the scheduled arrival --
// not the actual submit -- to the completion, so a late generator cannot
// hide queueing (no coordinated omission).
qldpc_status qldpc_server_loadgen(qldpc_server srv, const qldpc_loadgen_config *lg, qldpc_loadgen_result *res,
                                  double *lat_us, int64_t lat_cap) {
    if (!srv || !lg || !res || lg->rate_shots_per_s <= 0 || lg->duration_s <= 0 || lg->ncodes != (int32_t)srv->codes.size())
        return set_error(QLDPC_ERR_INVALID_ARG, "server_loadgen: bad arguments");
    const int32_t nc = lg->ncodes;
    for (int c = 0; c < nc; ++c)
        if (!lg->pool_syn[c] || !lg->pool_prior[c] || lg->pool_size[c] < 64)
            return set_error(QLDPC_ERR_INVALID_ARG, "server_loadgen: each pool needs >= 64 shots");
    std::mt19937_64 rng(lg->seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const double mean_shots = lg->p_single * 1.0 + (1.0 - lg->p_single) * 64.0;
    const double mean_gap_s = mean_shots / lg->rate_shots_per_s;
    // output ring for outstanding requests
    const int64_t ring = (int64_t)srv->cfg.queue_capacity + (int64_t)srv->slots.size() * srv->cfg.max_batch_shots + 16;
    std::vector<uint32_t> out_err((size_t)ring * 64 * srv->max_ew);
    std::vector<uint8_t> out_conv((size_t)ring * 64), out_it((size_t)ring * 64);
    std::vector<int64_t> sched;                 // scheduled arrival per request id
    std::vector<int32_t> shots_of;
    std::vector<double> lat;
    lat.reserve(1 << 16);
    int64_t rejected = 0, shots_done = 0, outstanding = 0;
    std::vector<qldpc_completion> buf(4096);
    auto drain = [&]() -> qldpc_status {
        int32_t n = 0;
        qldpc_status st = qldpc_server_poll(srv, buf.data(), (int32_t)buf.size(), &n);
        if (st != QLDPC_OK && st != QLDPC_ERR_NOT_READY) return st;
        for (int32_t i = 0; i < n; ++i) {
            lat.push_back((buf[i].t_done_ns - sched[buf[i].req_id]) * 1e-3);
            shots_done += buf[i].nshots;
            --outstanding;
        }
        return QLDPC_OK;
    };
    const int64_t t0 = now_ns() + 1000000;   // start 1 ms from now
    const int64_t t_end = t0 + (int64_t)(lg->duration_s * 1e9);
    double t_next = (double)t0;
    uint64_t id = 0;
    qldpc_status st = QLDPC_OK;
    while (st == QLDPC_OK) {
        const int64_t arrive = (int64_t)t_next;
        if (arrive >= t_end) break;
        while (now_ns() < arrive) {
            st = drain();
            if (st != QLDPC_OK) break;
        }
        const int32_t c = (int32_t)(U(rng) * nc) % nc;
        const int32_t ns = U(rng) < lg->p_single ? 1 : 64;
        const int32_t dec = (srv->weights[c] && U(rng) < lg->p_neural) ? 1 : 0;
        const int32_t start = (int32_t)(U(rng) * (lg->pool_size[c] - ns + 1));
        const qldpc_code cc = srv->codes[c];
        const int32_t sw = (cc->m + 31) / 32;
        const int64_t slot = (int64_t)(id % (uint64_t)ring);
        sched.push_back(arrive);
        shots_of.push_back(ns);
        qldpc_status s2 = qldpc_server_submit(srv, c, dec, ns, lg->pool_syn[c] + (size_t)start * sw,
                                              lg->pool_prior[c] + start, out_err.data() + (size_t)slot * 64 * srv->max_ew,
                                              out_conv.data() + slot * 64, out_it.data() + slot * 64, id);
        if (s2 == QLDPC_ERR_CAPACITY) {
            ++rejected;
        } else if (s2 != QLDPC_OK) {
            st = s2;
            break;
        } else {
            ++outstanding;
        }
        ++id;
        t_next += -std::log(1.0 - U(rng)) * mean_gap_s * 1e9;
    }
    const int64_t t_stop_arrivals = now_ns();
    // wait for the rest (bounded)
    const int64_t deadline = now_ns() + 30LL * 1000000000LL;
    while (st == QLDPC_OK && outstanding > 0 && now_ns() < deadline) {
        st = drain();
        std::this_thread::yield();
    }
    if (st != QLDPC_OK) return st;
    if (outstanding > 0) return set_error(QLDPC_ERR_DEVICE, "server_loadgen: requests did not complete in 30 s");
    const int64_t t_last = now_ns();
    std::vector<double> sorted = lat;
    std::sort(sorted.begin(), sorted.end());
    auto pct = [&](double q) { return sorted.empty() ? 0.0 : sorted[(size_t)std::min<double>(sorted.size() - 1, q * sorted.size())]; };
    res->requests = (int64_t)lat.size();
    res->shots = shots_done;
    res->rejected = rejected;
    res->wall_s = (t_last - t0) * 1e-9;
    res->offered_s = (t_stop_arrivals - t0) * 1e-9;
    res->p50_us = pct(0.50);
    res->p99_us = pct(0.99);
    res->p999_us = pct(0.999);
    double sum = 0;
    for (double v : lat) sum += v;
    res->mean_us = lat.empty() ? 0 : sum / lat.size();
    res->max_us = sorted.empty() ? 0 : sorted.back();
    res->shots_per_s = shots_done / std::max(1e-9, res->wall_s);
    if (lat_us)
        for (int64_t i = 0; i < std::min<int64_t>(lat_cap, (int64_t)lat.size()); ++i) lat_us[i] = lat[i];
    return QLDPC_OK;
}

}  // extern "C"
