// Host runtime of the decoder library: C ABI, code objects, validation and
// kernel selection.  A code object holds the Tanner graph of H (Section 2:
// the sets S_v(m), S_c(n)) in one of two device forms, uploaded once at
// creation: for a lifted-product code with a compiled block pattern only the
// circulant shifts of its blocks; for any other H its edge lists (CSR for
// the check pass, CSC positions for the variable pass).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include <fstream>
#include <sstream>

#include "internal.h"
#include "shapes.h"

using namespace qldpc;

namespace {
thread_local std::string g_err;
}  // namespace

namespace qldpc {

qldpc_status set_error(qldpc_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

qldpc_status hip_error(hipError_t e, const char *what) {
    return set_error(QLDPC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace qldpc

namespace {
qldpc_status fail(qldpc_status st, const std::string &msg) { return set_error(st, msg); }
qldpc_status hip_fail(hipError_t e, const char *what) { return hip_error(e, what); }

// Messages in registers: a wavefront per 64 / L shots for L <= 64 (both
// schedules), a workgroup of L / 64 wavefronts per shot for L = 128, 256,
// 512 (flooding).
bool reg_supported(const qldpc_code_s *code, int sched) {
    if (code->L <= 0) return false;
    if (code->L <= 64) return true;
    return (code->L == 128 || code->L == 256 || code->L == 512) && sched == QLDPC_FLOOD;
}
}  // namespace

namespace qldpc {

qldpc_status prepare_decode(qldpc_code code, const qldpc_decode_params *p, int32_t batch, LaunchKey *key,
                            DecodeArgs *a) {
    if (!code || !p) return fail(QLDPC_ERR_INVALID_ARG, "decode: null code or params");
    if (batch < 0) return fail(QLDPC_ERR_INVALID_ARG, "decode: negative batch");
    if (p->max_iters < 1 || p->max_iters > 255)
        return fail(QLDPC_ERR_INVALID_ARG, "decode: max_iters must be in [1, 255]");
    if (p->fmt != QLDPC_F32 && p->fmt != QLDPC_I8Q4 && p->fmt != QLDPC_I16Q8)
        return fail(QLDPC_ERR_INVALID_ARG, "decode: bad format");
    if (p->sched != QLDPC_FLOOD && p->sched != QLDPC_LAYERED)
        return fail(QLDPC_ERR_INVALID_ARG, "decode: bad schedule");
    if (p->prior_mode != QLDPC_PRIOR_PER_SHOT && p->prior_mode != QLDPC_PRIOR_PER_BIT)
        return fail(QLDPC_ERR_INVALID_ARG, "decode: bad prior mode");
    if (!(p->alpha > 0.0f && p->alpha <= 1.0f)) return fail(QLDPC_ERR_INVALID_ARG, "decode: alpha must be in (0, 1]");
    if (p->layout < QLDPC_LAYOUT_AUTO || p->layout > QLDPC_LAYOUT_HBM)
        return fail(QLDPC_ERR_INVALID_ARG, "decode: bad layout");
    if (p->waves_per_shot != 0 && p->waves_per_shot != 8 && p->waves_per_shot != 16)
        return fail(QLDPC_ERR_INVALID_ARG, "decode: waves_per_shot must be 0, 8 or 16");
    *a = DecodeArgs{};
    a->code = code->dev;
    a->batch = batch;
    a->max_iters = p->max_iters;
    a->early_stop = p->early_stop ? 1 : 0;
    a->alpha = p->alpha;
    if (p->fmt != QLDPC_F32) {
        int sh = 0;
        for (; sh <= 8; ++sh) {
            const float num = p->alpha * (float)(1 << sh);
            if (num == std::floor(num)) break;
        }
        if (sh > 8) return fail(QLDPC_ERR_UNSUPPORTED, "decode: integer formats need alpha = num / 2^s, s <= 8");
        a->alpha_num = (int32_t)(p->alpha * (float)(1 << sh));
        a->alpha_shift = sh;
    }
    *key = LaunchKey{};
    key->which = code->which;
    key->L = code->L;
    key->fmt = p->fmt;
    key->sched = p->sched;
    key->per_bit = p->prior_mode == QLDPC_PRIOR_PER_BIT;
    if (code->L == 0) {
        // edge-list decoder: flooding, one wavefront per shot, messages in LDS
        a->code = nullptr;
        if (p->sched != QLDPC_FLOOD)
            return fail(QLDPC_ERR_UNSUPPORTED, "decode: the layered schedule needs quasi-cyclic lift data");
        if (p->layout != QLDPC_LAYOUT_AUTO && p->layout != QLDPC_LAYOUT_WAVE)
            return fail(QLDPC_ERR_UNSUPPORTED, "decode: a code without a compiled block pattern has one layout "
                                               "(wavefront per shot)");
        const int b = p->fmt == QLDPC_F32 ? 4 : p->fmt == QLDPC_I16Q8 ? 2 : 1;
        if (gen_lds_bytes(code->m, code->n, code->max_dc, b) > kGenMaxLds)
            return fail(QLDPC_ERR_UNSUPPORTED, "decode: the edge messages of this code do not fit one wavefront's "
                                               "LDS in this format");
        key->layout = QLDPC_LAYOUT_WAVE;
        key->nw = 0;
        return QLDPC_OK;
    }
    const bool block_ok = p->sched == QLDPC_FLOOD && code->L >= 64;
    int layout = p->layout, nw = p->waves_per_shot;
    // L = 256, 512: L / 64 register wavefronts per shot (FP32 flooding at L = 256,
    // 8192 shots, p = 0.03: 3.9 M syndromes/s against 1.03 M with messages in
    // HBM; L = 512, 4096 shots: 0.96 M against 0.35 M); layered decoding has
    // neither layout there
    if (layout == QLDPC_LAYOUT_AUTO && code->L > 128)
        layout = p->sched == QLDPC_FLOOD ? QLDPC_LAYOUT_WAVE_REG : QLDPC_LAYOUT_HBM;
    if (layout == QLDPC_LAYOUT_AUTO) {
        bool found = false;
        {
            std::lock_guard<std::mutex> g(code->tune_mu);
            auto it = code->tune.find(tune_key(p->fmt, p->sched, p->prior_mode, size_class(batch)));
            if (it != code->tune.end()) {
                layout = it->second.layout;
                if (nw == 0) nw = it->second.nw;
                found = true;
            }
        }
        // Defaults measured on MI355X (65536 shots at L = 64, 32768 at L = 128,
        // p = 0.01 / 0.03 / 0.05): messages in registers (L = 64 FP32 flooding
        // 38.8 M syndromes/s against 26.9 M for 8-wave workgroups; L = 128
        // flooding, two wavefronts per shot, 13.0 M FP32 / 12.8 M int8 against
        // 12.0 / 8.6 M for 8-wave workgroups with messages in LDS and 3.3 /
        // 4.55 M with messages in HBM); L = 128 layered a wavefront per shot;
        // small batches (latency) 16-wave workgroups.
        const bool reg_ok = reg_supported(code, p->sched);
        if (!found) {
            if (block_ok && batch < 512) {
                layout = QLDPC_LAYOUT_BLOCK;
                if (nw == 0) nw = batch < 512 ? 16 : 8;
            } else {
                layout = reg_ok ? QLDPC_LAYOUT_WAVE_REG : QLDPC_LAYOUT_WAVE;
            }
        }
    }
    if (layout == QLDPC_LAYOUT_BLOCK) {
        if (!block_ok)
            return fail(QLDPC_ERR_UNSUPPORTED, "decode: the workgroup layout needs flooding and L >= 64");
        if (nw == 0) nw = 16;
    }
    if (layout == QLDPC_LAYOUT_WAVE_REG && !reg_supported(code, p->sched))
        return fail(QLDPC_ERR_UNSUPPORTED, "decode: register-resident messages need L <= 64, or flooding with "
                                           "L in {128, 256, 512} (L / 64 wavefronts per shot)");
    if (layout == QLDPC_LAYOUT_HBM && (p->sched != QLDPC_FLOOD || code->L < 128))
        return fail(QLDPC_ERR_UNSUPPORTED, "decode: the HBM layout needs flooding and L in {128, 256, 512}");
    if (layout != QLDPC_LAYOUT_HBM && layout != QLDPC_LAYOUT_WAVE_REG && code->L > 128)
        return fail(QLDPC_ERR_UNSUPPORTED, "decode: lifts above 128 keep messages in registers "
                                           "(QLDPC_LAYOUT_WAVE_REG, flooding) or in HBM (QLDPC_LAYOUT_HBM)");
    key->layout = layout;
    key->nw = nw;
    return QLDPC_OK;
}

}  // namespace qldpc

namespace {

// A code object over the edge lists of a validated CSR: row_ptr, col_idx,
// and for each variable its edges in increasing check order as LDS slots
// j * m + r of the edge-list decoder.  Refused (UNSUPPORTED) when its
// messages would not fit one wavefront's LDS even in int8.
qldpc_status create_generic(const qldpc_code_desc *d, int32_t max_dc, int32_t max_dv, int32_t device,
                            qldpc_code *out) {
    const int32_t m = d->m, n = d->n, nnz = d->row_ptr[d->m];
    if (gen_lds_bytes(m, n, max_dc, 1) > kGenMaxLds)
        return fail(QLDPC_ERR_UNSUPPORTED, "code_create: code too large for the edge-list decoder (messages of "
                                           "max check degree x checks must fit 64 KB of LDS in int8)");
    std::vector<int32_t> col_ptr(n + 1, 0), vn_slot(nnz);
    for (int32_t f = 0; f < nnz; ++f) col_ptr[d->col_idx[f] + 1]++;
    for (int32_t c = 0; c < n; ++c) col_ptr[c + 1] += col_ptr[c];
    std::vector<int32_t> fill(col_ptr.begin(), col_ptr.end() - 1);
    for (int32_t r = 0; r < m; ++r)   // rows in increasing order: each column's list is sorted by row
        for (int32_t f = d->row_ptr[r]; f < d->row_ptr[r + 1]; ++f)
            vn_slot[fill[d->col_idx[f]]++] = (f - d->row_ptr[r]) * m + r;
    auto *code = new (std::nothrow) qldpc_code_s();
    if (!code) return fail(QLDPC_ERR_OUT_OF_MEMORY, "code_create: host allocation failed");
    code->m = m;
    code->n = n;
    code->nnz = nnz;
    code->max_dc = max_dc;
    code->max_dv = max_dv;
    code->L = 0;
    code->which = -1;
    code->device = device;
    const size_t words = (size_t)(m + 1) + nnz + (n + 1) + nnz;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) { delete code; return hip_fail(e, "hipGetDevice"); }
    e = hipSetDevice(device);
    if (e != hipSuccess) { delete code; return hip_fail(e, "hipSetDevice"); }
    e = hipMalloc(&code->gen_mem, words * sizeof(int32_t));
    if (e != hipSuccess) {
        (void)hipSetDevice(prev);
        delete code;
        return fail(QLDPC_ERR_OUT_OF_MEMORY, "code_create: hipMalloc failed");
    }
    int32_t *base = static_cast<int32_t *>(code->gen_mem);
    GenCode &g = code->gen;
    g.m = m;
    g.n = n;
    g.nnz = nnz;
    g.max_dc = max_dc;
    g.row_ptr = base;
    g.col_idx = base + (m + 1);
    g.col_ptr = base + (m + 1) + nnz;
    g.vn_slot = base + (m + 1) + nnz + (n + 1);
    std::vector<int32_t> host;
    host.reserve(words);
    host.insert(host.end(), d->row_ptr, d->row_ptr + m + 1);
    host.insert(host.end(), d->col_idx, d->col_idx + nnz);
    host.insert(host.end(), col_ptr.begin(), col_ptr.end());
    host.insert(host.end(), vn_slot.begin(), vn_slot.end());
    e = hipMemcpy(code->gen_mem, host.data(), words * sizeof(int32_t), hipMemcpyHostToDevice);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipFree(code->gen_mem);
        delete code;
        return hip_fail(e, "code_create: upload");
    }
    *out = code;
    return QLDPC_OK;
}

}  // namespace

namespace qldpc {

hipError_t launch_code_decode(qldpc_code code, const LaunchKey &k, const DecodeArgs &a, hipStream_t stream) {
    if (code->L == 0) return launch_generic_decode(code->gen, k, a, stream);
    return launch_decode(k, a, stream);
}

}  // namespace qldpc

extern "C" {

const char *qldpc_last_error(void) { return g_err.c_str(); }

int32_t qldpc_version(void) { return 100; }

void qldpc_default_params(qldpc_decode_params *p) {
    if (!p) return;
    p->fmt = QLDPC_F32;
    p->sched = QLDPC_FLOOD;
    p->alpha = 0.75f;
    p->max_iters = 32;
    p->early_stop = 1;
    p->prior_mode = QLDPC_PRIOR_PER_SHOT;
    p->layout = QLDPC_LAYOUT_AUTO;
    p->waves_per_shot = 0;
}

qldpc_status qldpc_quantize_prior(const float *llr, int8_t *out, int64_t count) {
    if (count < 0 || (count > 0 && (!llr || !out))) return fail(QLDPC_ERR_INVALID_ARG, "quantize_prior: bad arguments");
    for (int64_t i = 0; i < count; ++i) {
        const float v = llr[i] * 16.0f;   // exact: scaling by a power of two
        double r = std::floor(std::fabs((double)v) + 0.5);
        if (v < 0) r = -r;
        if (r > 127) r = 127;
        if (r < -127) r = -127;
        out[i] = (int8_t)r;
    }
    return QLDPC_OK;
}

qldpc_status qldpc_quantize_prior_q8(const float *llr, int16_t *out, int64_t count) {
    if (count < 0 || (count > 0 && (!llr || !out)))
        return fail(QLDPC_ERR_INVALID_ARG, "quantize_prior_q8: bad arguments");
    for (int64_t i = 0; i < count; ++i) {
        const float v = llr[i] * 256.0f;   // exact: scaling by a power of two
        double r = std::floor(std::fabs((double)v) + 0.5);
        if (v < 0) r = -r;
        if (r > 32767) r = 32767;
        if (r < -32767) r = -32767;
        out[i] = (int16_t)r;
    }
    return QLDPC_OK;
}

qldpc_status qldpc_code_create(const qldpc_code_desc *d, int32_t device, qldpc_code *out) {
    if (!d || !out) return fail(QLDPC_ERR_INVALID_ARG, "code_create: null argument");
    if (d->m <= 0 || d->n <= 0 || !d->row_ptr || !d->col_idx)
        return fail(QLDPC_ERR_INVALID_ARG, "code_create: empty matrix or null CSR");
    if (d->row_ptr[0] != 0) return fail(QLDPC_ERR_INVALID_ARG, "code_create: row_ptr[0] != 0");
    int32_t max_dc = 0;
    std::vector<int32_t> coldeg(d->n, 0);
    for (int32_t r = 0; r < d->m; ++r) {
        const int32_t lo = d->row_ptr[r], hi = d->row_ptr[r + 1];
        if (hi < lo) return fail(QLDPC_ERR_INVALID_ARG, "code_create: row_ptr not monotone");
        if (hi - lo < 2)
            return fail(QLDPC_ERR_INVALID_ARG, "code_create: check " + std::to_string(r) + " has degree < 2");
        for (int32_t f = lo; f < hi; ++f) {
            const int32_t c = d->col_idx[f];
            if (c < 0 || c >= d->n) return fail(QLDPC_ERR_INVALID_ARG, "code_create: column out of range");
            if (f > lo && c <= d->col_idx[f - 1])
                return fail(QLDPC_ERR_INVALID_ARG, "code_create: columns not strictly increasing");
            coldeg[c]++;
        }
        if (hi - lo > max_dc) max_dc = hi - lo;
    }
    int32_t max_dv = 0;
    for (int32_t c = 0; c < d->n; ++c) max_dv = std::max(max_dv, coldeg[c]);

    if (d->lift_L <= 0 || !d->base_exp) return create_generic(d, max_dc, max_dv, device, out);
    const int32_t L = d->lift_L, bm = d->base_m, bn = d->base_n;
    if (bm <= 0 || bn <= 0 || (int64_t)bm * L != d->m || (int64_t)bn * L != d->n)
        return fail(QLDPC_ERR_INVALID_ARG, "code_create: lift dimensions disagree with m, n");
    for (int32_t i = 0; i < bm * bn; ++i)
        if (d->base_exp[i] < -1 || d->base_exp[i] >= L)
            return fail(QLDPC_ERR_INVALID_ARG, "code_create: base exponent out of [-1, L)");
    // the CSR must equal the expansion of the lift
    for (int32_t R = 0; R < bm; ++R)
        for (int32_t t = 0; t < L; ++t) {
            const int32_t r = R * L + t;
            std::vector<int32_t> want;
            for (int32_t C = 0; C < bn; ++C) {
                const int32_t a = d->base_exp[R * bn + C];
                if (a >= 0) want.push_back(C * L + (t + a) % L);
            }
            const int32_t lo = d->row_ptr[r], hi = d->row_ptr[r + 1];
            if ((int32_t)want.size() != hi - lo)
                return fail(QLDPC_ERR_INVALID_ARG, "code_create: CSR disagrees with the lift (row " + std::to_string(r) + ")");
            for (int32_t f = lo; f < hi; ++f)
                if (d->col_idx[f] != want[f - lo])
                    return fail(QLDPC_ERR_INVALID_ARG, "code_create: CSR disagrees with the lift (row " + std::to_string(r) + ")");
        }
    // match a compiled block pattern
    int which = -1;
    if (bm == 15 && bn == 34) {
        for (int w = 0; w < 2 && which < 0; ++w) {
            bool ok = true;
            for (int32_t R = 0; R < bm && ok; ++R)
                for (int32_t C = 0; C < bn && ok; ++C)
                    ok = (d->base_exp[R * bn + C] >= 0) == lp35_nonzero(w, R, C);
            if (ok) which = w;
        }
    }
    // a valid lift without a compiled block pattern or lift size: edge lists
    if (which < 0 || (L != 16 && L != 32 && L != 64 && L != 128 && L != 256 && L != 512))
        return create_generic(d, max_dc, max_dv, device, out);

    auto *code = new (std::nothrow) qldpc_code_s();
    if (!code) return fail(QLDPC_ERR_OUT_OF_MEMORY, "code_create: host allocation failed");
    code->m = d->m;
    code->n = d->n;
    code->nnz = d->row_ptr[d->m];
    code->max_dc = max_dc;
    code->max_dv = max_dv;
    code->L = L;
    code->which = which;
    code->device = device;
    DevCode host{};
    const PatternTables &T = which == 0 ? ShapeLP35Z::T : ShapeLP35X::T;
    for (int R = 0; R < 15; ++R)
        for (int j = 0; j < 8; ++j) {
            const int32_t s = d->base_exp[R * bn + T.slot_bc[R][j]];
            host.shift[R * 8 + j] = s;
            uint64_t low = 0;
            if (L < 64) {
                const uint64_t seg = (1ull << (L - s)) - 1ull;
                for (int g = 0; g < 64 / L; ++g) low |= seg << (g * L);
            }
            host.lowmask[R * 8 + j] = low;
        }
    for (int C = 0; C < T.ncols(); ++C)
        for (int i = 0; i < T.col_deg[C]; ++i) {
            const int slot = T.col_R[C][i] * 8 + T.col_j[C][i];
            const int32_t s = host.shift[slot], c = (L - s) % L;
            host.colrot[C][i] = ColRot{s, c, 4 * c, 4 * s, host.lowmask[slot], 0};
        }
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) { delete code; return hip_fail(e, "hipGetDevice"); }
    e = hipSetDevice(device);
    if (e != hipSuccess) { delete code; return hip_fail(e, "hipSetDevice"); }
    e = hipMalloc(&code->dev, sizeof(DevCode));
    if (e != hipSuccess) {
        (void)hipSetDevice(prev);
        delete code;
        return fail(QLDPC_ERR_OUT_OF_MEMORY, "code_create: hipMalloc failed");
    }
    e = hipMemcpy(code->dev, &host, sizeof(DevCode), hipMemcpyHostToDevice);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        (void)hipFree(code->dev);
        delete code;
        return hip_fail(e, "code_create: upload");
    }
    *out = code;
    return QLDPC_OK;
}

qldpc_status qldpc_code_destroy(qldpc_code code) {
    if (!code) return QLDPC_OK;
    if (code->dev) (void)hipFree(code->dev);
    if (code->gen_mem) (void)hipFree(code->gen_mem);
    delete code;
    return QLDPC_OK;
}

qldpc_status qldpc_code_info(qldpc_code c, int32_t *m, int32_t *n, int32_t *nnz, int32_t *max_dc,
                             int32_t *max_dv) {
    if (!c) return fail(QLDPC_ERR_INVALID_ARG, "code_info: null code");
    if (m) *m = c->m;
    if (n) *n = c->n;
    if (nnz) *nnz = c->nnz;
    if (max_dc) *max_dc = c->max_dc;
    if (max_dv) *max_dv = c->max_dv;
    return QLDPC_OK;
}

namespace {

// Bytes of message workspace for key k and `batch` shots (0 when on chip).
size_t workspace_bytes_for(const qldpc_code code, const LaunchKey &k, int32_t batch) {
    if (k.layout != QLDPC_LAYOUT_HBM) return 0;
    const size_t bytes_per_msg = k.fmt == QLDPC_F32 ? 4 : k.fmt == QLDPC_I16Q8 ? 2 : 1;
    return (size_t)batch * 120 * (size_t)code->L * bytes_per_msg;
}

qldpc_status decode_impl(qldpc_code code, const qldpc_decode_params *p, int32_t batch, const uint32_t *syn,
                         const void *priors, uint32_t *err, uint8_t *conv, uint8_t *iters, float *post, bool with_ws,
                         void *ws, size_t ws_bytes, void *stream, const char *who) {
    LaunchKey k{};
    DecodeArgs a{};
    qldpc_status st = prepare_decode(code, p, batch, &k, &a);
    if (st != QLDPC_OK || batch == 0) return st;
    if (!syn || !priors || !err || !conv) return fail(QLDPC_ERR_INVALID_ARG, std::string(who) + ": null buffer");
    const size_t need = workspace_bytes_for(code, k, batch);
    if (need > 0) {
        if (!with_ws)
            return fail(QLDPC_ERR_UNSUPPORTED, std::string(who) +
                                                   ": this layout keeps messages in a device workspace; use "
                                                   "qldpc_decode_batch_ws");
        if (!ws || ws_bytes < need || ((uintptr_t)ws & 255) != 0)
            return fail(QLDPC_ERR_INVALID_ARG, std::string(who) + ": workspace missing, too small or not 256-byte aligned");
    }
    a.syn = syn;
    a.prior = priors;
    a.err = err;
    a.conv = conv;
    a.iters = iters;
    a.post = post;
    k.post = post != nullptr;
    const hipError_t e = k.layout == QLDPC_LAYOUT_HBM ? launch_hbm_decode(k, a, ws, (hipStream_t)stream)
                                                      : launch_code_decode(code, k, a, (hipStream_t)stream);
    if (e == hipErrorNotSupported)
        return fail(QLDPC_ERR_UNSUPPORTED, std::string(who) + ": no kernel for this format/schedule/layout/L");
    if (e != hipSuccess) return hip_fail(e, "decode launch");
    return QLDPC_OK;
}

}  // namespace

qldpc_status qldpc_decode_batch(qldpc_code code, const qldpc_decode_params *p, int32_t batch,
                                const uint32_t *syn, const void *priors, uint32_t *err,
                                uint8_t *conv, uint8_t *iters, float *post, void *stream) {
    return decode_impl(code, p, batch, syn, priors, err, conv, iters, post, false, nullptr, 0, stream, "decode_batch");
}

qldpc_status qldpc_decode_workspace_bytes(qldpc_code code, const qldpc_decode_params *p, int32_t batch,
                                          size_t *bytes) {
    if (!bytes) return fail(QLDPC_ERR_INVALID_ARG, "decode_workspace_bytes: null output");
    LaunchKey k{};
    DecodeArgs a{};
    qldpc_status st = prepare_decode(code, p, batch, &k, &a);
    if (st != QLDPC_OK) return st;
    *bytes = workspace_bytes_for(code, k, batch);
    return QLDPC_OK;
}

qldpc_status qldpc_decode_batch_ws(qldpc_code code, const qldpc_decode_params *p, int32_t batch,
                                   const uint32_t *syn, const void *priors, uint32_t *err, uint8_t *conv,
                                   uint8_t *iters, float *post, void *workspace, size_t workspace_bytes,
                                   void *stream) {
    return decode_impl(code, p, batch, syn, priors, err, conv, iters, post, true, workspace, workspace_bytes, stream,
                       "decode_batch_ws");
}

qldpc_status qldpc_autotune(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                            const uint32_t *syn, const void *priors, uint32_t *err, uint8_t *conv,
                            uint8_t *iters, void *stream, qldpc_decode_params *best) {
    if (!code || !params || !best) return fail(QLDPC_ERR_INVALID_ARG, "autotune: null argument");
    if (batch <= 0) return fail(QLDPC_ERR_INVALID_ARG, "autotune: batch must be positive");
    if (!syn || !priors || !err || !conv) return fail(QLDPC_ERR_INVALID_ARG, "autotune: null buffer");
    if (code->L > 128)
        return fail(QLDPC_ERR_UNSUPPORTED, "autotune: lifts above 128 have one layout without a workspace "
                                           "(messages in registers, AUTO's choice)");
    struct Cand { int layout, nw; };
    std::vector<Cand> cands = {{QLDPC_LAYOUT_WAVE, 0}};
    if (reg_supported(code, params->sched)) cands.push_back({QLDPC_LAYOUT_WAVE_REG, 0});
    if (params->sched == QLDPC_FLOOD && code->L >= 64) {
        cands.push_back({QLDPC_LAYOUT_BLOCK, 8});
        cands.push_back({QLDPC_LAYOUT_BLOCK, 16});
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    hipError_t he = hipEventCreate(&e0);
    if (he != hipSuccess) return hip_fail(he, "autotune: event");
    he = hipEventCreate(&e1);
    if (he != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(he, "autotune: event"); }
    TuneChoice bestc{};
    bestc.ms = 1e30f;
    qldpc_status rc = QLDPC_OK;
    for (const Cand &c : cands) {
        qldpc_decode_params q = *params;
        q.layout = c.layout;
        q.waves_per_shot = c.nw;
        rc = qldpc_decode_batch(code, &q, batch, syn, priors, err, conv, iters, nullptr, stream);  // warm-up
        if (rc != QLDPC_OK) break;
        const int reps = 3;
        he = hipEventRecord(e0, st);
        if (he != hipSuccess) { rc = hip_fail(he, "autotune: record"); break; }
        for (int r = 0; r < reps && rc == QLDPC_OK; ++r)
            rc = qldpc_decode_batch(code, &q, batch, syn, priors, err, conv, iters, nullptr, stream);
        he = hipEventRecord(e1, st);
        if (rc != QLDPC_OK) break;
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) { rc = hip_fail(he, "autotune: timing"); break; }
        ms /= reps;
        if (ms < bestc.ms) bestc = TuneChoice{c.layout, c.nw, ms};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != QLDPC_OK) return rc;
    {
        std::lock_guard<std::mutex> g(code->tune_mu);
        code->tune[tune_key(params->fmt, params->sched, params->prior_mode, size_class(batch))] = bestc;
    }
    *best = *params;
    best->layout = bestc.layout;
    best->waves_per_shot = bestc.nw;
    return QLDPC_OK;
}

qldpc_status qldpc_tune_save(qldpc_code code, const char *path) {
    if (!code || !path) return fail(QLDPC_ERR_INVALID_ARG, "tune_save: null argument");
    std::ostringstream o;
    o << "{\"L\": " << code->L << ", \"pattern\": " << code->which << ", \"entries\": [";
    {
        std::lock_guard<std::mutex> g(code->tune_mu);
        bool first = true;
        for (const auto &kv : code->tune) {
            o << (first ? "" : ", ") << "[" << kv.first << ", " << kv.second.layout << ", "
              << kv.second.nw << ", " << kv.second.ms << "]";
            first = false;
        }
    }
    o << "]}\n";
    std::ofstream f(path);
    if (!f) return fail(QLDPC_ERR_INVALID_ARG, std::string("tune_save: cannot write ") + path);
    f << o.str();
    return QLDPC_OK;
}

qldpc_status qldpc_tune_load(qldpc_code code, const char *path) {
    if (!code || !path) return fail(QLDPC_ERR_INVALID_ARG, "tune_load: null argument");
    std::ifstream f(path);
    if (!f) return fail(QLDPC_ERR_INVALID_ARG, std::string("tune_load: cannot read ") + path);
    std::stringstream buf;
    buf << f.rdbuf();
    std::string t = buf.str();
    for (char &ch : t)
        if (ch == '[' || ch == ']' || ch == '{' || ch == '}' || ch == ',' || ch == ':' || ch == '"') ch = ' ';
    std::istringstream in(t);
    std::string tok;
    int L = -1, pattern = -1;
    std::vector<double> nums;
    while (in >> tok) {
        if (tok == "L") in >> L;
        else if (tok == "pattern") in >> pattern;
        else if (tok == "entries") {
            double v;
            while (in >> v) nums.push_back(v);
        }
    }
    if (L < 0 || pattern < -1 || nums.size() % 4 != 0) return fail(QLDPC_ERR_INVALID_ARG, "tune_load: malformed file");
    if (L != code->L || pattern != code->which) return QLDPC_OK;   // for another code
    std::lock_guard<std::mutex> g(code->tune_mu);
    for (size_t i = 0; i < nums.size(); i += 4) {
        const int layout = (int)nums[i + 1], nw = (int)nums[i + 2];
        if (layout != QLDPC_LAYOUT_WAVE && layout != QLDPC_LAYOUT_BLOCK && layout != QLDPC_LAYOUT_WAVE_REG) continue;
        if (layout == QLDPC_LAYOUT_BLOCK && nw != 8 && nw != 16) continue;
        const int key = (int)nums[i];
        if (layout == QLDPC_LAYOUT_WAVE_REG && !reg_supported(code, (key / 16) % 2)) continue;   // key: tune_key
        code->tune[key] = TuneChoice{layout, nw, (float)nums[i + 3]};
    }
    return QLDPC_OK;
}

}  // extern "C"
