// Continuous-batching decode server (the paper's proposal of several
// asynchronous decoders overlapping transfers and kernels, Table 1 and
// Section 3, realised as a request loop).
//
// Requests (1..max_batch_shots syndromes of one code, plain or neural
// min-sum) enter a bounded queue.  A scheduler thread owns a fixed set of
// slots -- device buffers, pinned staging, a stream and a mixed-code plan
// each -- whose number is set by the HBM budget.  Whenever a slot is free it
// admits queued requests (FIFO, up to the slot's shot capacity) as one
// micro-batch: one copy-in of the packed inputs; for the plain min-sum shots
// one single-code decode per code (small micro-batches) or one mixed-code
// persistent decode (large ones with several codes); one neural decode per
// code for the neural shots; one copy-out of the packed outputs; an
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
    // One input and one output block per slot, packed per micro-batch so
    // that a micro-batch moves with one copy each way (see launch_slot).
    unsigned char *d_in = nullptr, *h_in = nullptr, *d_out = nullptr, *h_out = nullptr;
    uint8_t *d_used = nullptr;
    size_t o_conv = 0, o_iters = 0;       // output offsets of the launched micro-batch
    std::vector<int64_t> eoff;            // per shot: error-word offset in the output block
    std::vector<Request> reqs;
    bool busy = false;
    int32_t shots = 0;
};

}  // namespace

struct qldpc_server_s {
    qldpc_server_config cfg{};
    std::vector<qldpc_code> codes;
    std::vector<const float *> weights;
    int32_t max_sw = 0, max_ew = 0;
    std::vector<Slot> slots;
    // Light-load lane: one mapped-I/O session per code (null where none
    // could be made).  When nothing is in flight and the queue holds a single
    // small plain request, it is decoded at once through its code's session:
    // one launch reading and writing pinned host memory, no copies and no
    // micro-batch packing.
    std::vector<qldpc_session> fast;
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
    for (void *d : {(void *)s.d_in, (void *)s.d_out, (void *)s.d_used})
        if (d) (void)hipFree(d);
    for (void *h : {(void *)s.h_in, (void *)s.h_out})
        if (h) (void)hipHostFree(h);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    s = Slot{};
}

// Capacities of a slot's packed blocks for `shots` shots: inputs = priors,
// then the mixed-plan index arrays (code id, syndrome and error offsets),
// then the syndrome words; outputs = error words, flags, iterations.
size_t slot_in_bytes(int64_t shots, int32_t sw) { return (size_t)shots * (4 + 4 + 8 + 8 + 4 * (size_t)sw) + 16; }
size_t slot_out_bytes(int64_t shots, int32_t ew) { return (size_t)shots * (4 * (size_t)ew + 2) + 16; }

// Device bytes one slot holds for `shots` shots.
size_t slot_device_bytes(int64_t shots, int32_t sw, int32_t ew) {
    return slot_in_bytes(shots, sw) + slot_out_bytes(shots, ew) + (size_t)shots + 4 * ((size_t)shots + 17);
}

inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }

// Micro-batches of at most this many plain min-sum shots decode with one
// single-code launch per code present; larger ones through the mixed-code
// persistent plan (three bucketing kernels and a persistent grid per lift
// size, which pay off only on large batches).
constexpr int32_t kDirectShots = 1024;

// Largest request the light-load lane takes (its sessions' capacity).
constexpr int32_t kFastShots = 64;

// Packs the slot's requests into its staging and launches the micro-batch:
// one host-to-device copy of the packed inputs, the decodes, one
// device-to-host copy of the packed outputs, an event.  Shots are ordered
// plain min-sum first, then neural, each grouped by code, so every code's
// shots of one decoder are contiguous.
qldpc_status launch_slot(qldpc_server srv, Slot &s) {
    if (++srv->launches == srv->fail_launch_at)
        return set_error(QLDPC_ERR_DEVICE, "server: injected launch failure");
    const int32_t nc = (int32_t)srv->codes.size();
    struct Group { int32_t first = -1, count = 0; int64_t sw0 = 0, ew0 = 0; };
    std::vector<Group> plain(nc), neural(nc);
    int32_t n = 0, n_plain = 0, plain_codes = 0;
    int64_t sw_at = 0, ew_at = 0;
    for (int32_t dcd = 0; dcd < 2; ++dcd)
        for (int32_t c = 0; c < nc; ++c)
            for (Request &r : s.reqs)
                if (r.decoder == dcd && r.code == c) {
                    Group &g = dcd == 0 ? plain[c] : neural[c];
                    if (g.first < 0) {
                        g.first = n;
                        g.sw0 = sw_at;
                        g.ew0 = ew_at;
                        if (dcd == 0) ++plain_codes;
                    }
                    const qldpc_code cc = srv->codes[c];
                    r.first_shot = n;
                    g.count += r.nshots;
                    n += r.nshots;
                    if (dcd == 0) n_plain += r.nshots;
                    sw_at += (int64_t)r.nshots * ((cc->m + 31) / 32);
                    ew_at += (int64_t)r.nshots * ((cc->n + 31) / 32);
                }
    const bool mixed = n_plain > kDirectShots && plain_codes > 1;
    const int32_t n_idx = mixed ? n_plain : 0;
    const size_t o_prior = 0, o_cid = o_prior + 4 * (size_t)n, o_soff = align8(o_cid + 4 * (size_t)n_idx),
                 o_eoff = o_soff + 8 * (size_t)n_idx, o_syn = o_eoff + 8 * (size_t)n_idx,
                 in_bytes = o_syn + 4 * (size_t)sw_at;
    float *h_prior = reinterpret_cast<float *>(s.h_in + o_prior);
    int32_t *h_cid = reinterpret_cast<int32_t *>(s.h_in + o_cid);
    int64_t *h_soff = reinterpret_cast<int64_t *>(s.h_in + o_soff);
    int64_t *h_eoff = reinterpret_cast<int64_t *>(s.h_in + o_eoff);
    uint32_t *h_syn = reinterpret_cast<uint32_t *>(s.h_in + o_syn);
    s.eoff.resize(n);
    for (Request &r : s.reqs) {
        const qldpc_code cc = srv->codes[r.code];
        const int32_t sw = (cc->m + 31) / 32, ew = (cc->n + 31) / 32;
        const Group &g = r.decoder == 0 ? plain[r.code] : neural[r.code];
        const int32_t k0 = r.first_shot - g.first;   // position inside its group
        for (int32_t i = 0; i < r.nshots; ++i) {
            const int32_t sh = r.first_shot + i;
            const int64_t so = g.sw0 + (int64_t)(k0 + i) * sw, eo = g.ew0 + (int64_t)(k0 + i) * ew;
            std::memcpy(h_syn + so, r.syn + (size_t)i * sw, sizeof(uint32_t) * sw);
            h_prior[sh] = r.prior[i];
            s.eoff[sh] = eo;
            if (mixed && r.decoder == 0) {
                h_cid[sh] = r.code;
                h_soff[sh] = so;
                h_eoff[sh] = eo;
            }
        }
    }
    s.shots = n;
    s.o_conv = 4 * (size_t)ew_at;
    s.o_iters = s.o_conv + (size_t)n;
    const size_t out_bytes = s.o_iters + (size_t)n;
    const float *d_prior = reinterpret_cast<const float *>(s.d_in + o_prior);
    const uint32_t *d_syn = reinterpret_cast<const uint32_t *>(s.d_in + o_syn);
    uint32_t *d_err = reinterpret_cast<uint32_t *>(s.d_out);
    uint8_t *d_conv = s.d_out + s.o_conv, *d_iters = s.d_out + s.o_iters;
    hipStream_t st = s.stream;
    hipError_t e = hipMemcpyAsync(s.d_in, s.h_in, in_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_error(e, "server: copy-in");
    qldpc_status rc = QLDPC_OK;
    if (mixed) {
        rc = qldpc_mixed_decode(s.plan, n_plain, reinterpret_cast<const int32_t *>(s.d_in + o_cid),
                                reinterpret_cast<const int64_t *>(s.d_in + o_soff),
                                reinterpret_cast<const int64_t *>(s.d_in + o_eoff), d_syn, d_prior, d_err, d_conv,
                                d_iters, st);
    } else {
        for (int32_t c = 0; c < nc && rc == QLDPC_OK; ++c) {
            const Group &g = plain[c];
            if (g.count == 0) continue;
            rc = qldpc_decode_batch(srv->codes[c], &srv->cfg.params, g.count, d_syn + g.sw0, d_prior + g.first,
                                    d_err + g.ew0, d_conv + g.first, d_iters + g.first, nullptr, st);
        }
    }
    for (int32_t c = 0; c < nc && rc == QLDPC_OK; ++c) {
        const Group &g = neural[c];
        if (g.count == 0) continue;
        rc = qldpc_nbp_decode(srv->codes[c], g.count, srv->cfg.nms_T, srv->weights[c], &srv->cfg.params,
                              d_syn + g.sw0, d_prior + g.first, d_err + g.ew0, d_conv + g.first,
                              d_iters + g.first, s.d_used + g.first, st);
    }
    if (rc != QLDPC_OK) return rc;
    e = hipMemcpyAsync(s.h_out, s.d_out, out_bytes, hipMemcpyDeviceToHost, st);
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
            const uint32_t *h_err = reinterpret_cast<const uint32_t *>(s.h_out);
            for (int32_t i = 0; i < r.nshots; ++i) {
                const int32_t sh = r.first_shot + i;
                if (r.err) std::memcpy(r.err + (size_t)i * ew, h_err + s.eoff[sh], sizeof(uint32_t) * ew);
                if (r.conv) r.conv[i] = s.h_out[s.o_conv + sh];
                if (r.iters) r.iters[i] = s.h_out[s.o_iters + sh];
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
        // light load: nothing in flight and one small plain request queued
        bool idle = true;
        for (Slot &s : srv->slots) idle = idle && !s.busy;
        if (idle && !srv->stop) {
            Request r{};
            bool have = false;
            {
                std::lock_guard<std::mutex> g(srv->mu);
                if (srv->pending.size() == 1) {
                    const Request &f = srv->pending.front();
                    if (f.decoder == 0 && f.nshots <= kFastShots && srv->fast[f.code]) {
                        r = f;
                        srv->pending.pop_front();
                        have = true;
                    }
                }
            }
            if (have) {
                srv->inflight_shots += r.nshots;
                qldpc_status rc = QLDPC_OK;
                if (++srv->launches == srv->fail_launch_at)
                    rc = set_error(QLDPC_ERR_DEVICE, "server: injected launch failure");
                else
                    rc = qldpc_session_decode(srv->fast[r.code], r.nshots, r.syn, r.prior, r.err, r.conv, r.iters);
                srv->inflight_shots -= r.nshots;
                if (rc != QLDPC_OK) fail_server(srv, rc, qldpc_last_error());
                std::lock_guard<std::mutex> g(srv->mu);
                srv->completions.push_back(completion_of(r, rc, now_ns()));
                continue;
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
        const size_t ib = slot_in_bytes(B, srv->max_sw), ob = slot_out_bytes(B, srv->max_ew);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = dev_alloc(&s.d_in, ib);
        if (e == hipSuccess) e = dev_alloc(&s.d_out, ob);
        if (e == hipSuccess) e = dev_alloc(&s.d_used, B);
        if (e == hipSuccess) e = host_alloc(&s.h_in, ib);
        if (e == hipSuccess) e = host_alloc(&s.h_out, ob);
        if (e != hipSuccess) break;
        rc = qldpc_mixed_create(cfg->codes, cfg->ncodes, &cfg->params, (int32_t)B, 0, &s.plan);
        if (rc != QLDPC_OK) break;
    }
    if (e != hipSuccess || rc != QLDPC_OK) {
        for (Slot &s : srv->slots) free_slot(s);
        delete srv;
        return e != hipSuccess ? set_error(QLDPC_ERR_OUT_OF_MEMORY, "server_create: slot allocation") : rc;
    }
    srv->fast.assign(cfg->ncodes, nullptr);
    for (int c = 0; c < cfg->ncodes; ++c)
        if (qldpc_session_create(cfg->codes[c], &cfg->params, kFastShots, QLDPC_IO_MAPPED, &srv->fast[c]) != QLDPC_OK)
            srv->fast[c] = nullptr;   // that code's small requests go through micro-batches
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
    for (qldpc_session f : srv->fast)
        if (f) (void)qldpc_session_destroy(f);
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
