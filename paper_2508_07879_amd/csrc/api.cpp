// Host runtime of the decoder library: C ABI, code objects, validation and
// kernel selection.  The Tanner graph of a code object is described by its
// quasi-cyclic lift (Section 2: H and its sets S_v(m), S_c(n)); the kernels
// need only the circulant shifts of each block, uploaded once at creation.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/qldpc.h"
#include "kernels.h"
#include "shapes.h"

using namespace qldpc;

namespace {

thread_local std::string g_err;

qldpc_status fail(qldpc_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

qldpc_status hip_fail(hipError_t e, const char *what) {
    return fail(QLDPC_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct qldpc_code_s {
    int32_t m = 0, n = 0, nnz = 0, max_dc = 0, max_dv = 0;
    int32_t L = 0, which = -1, device = 0;
    std::vector<int32_t> shift;    // per slot (R * 8 + j)
    DevCode *dev = nullptr;        // device copy of the shift tables
};

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

    if (d->lift_L <= 0 || !d->base_exp)
        return fail(QLDPC_ERR_UNSUPPORTED, "code_create: the device kernels need quasi-cyclic lift data");
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
    if (which < 0)
        return fail(QLDPC_ERR_UNSUPPORTED,
                    "code_create: block pattern is not a 3x5 lifted-product H_Z or H_X pattern");
    if (L != 16 && L != 32 && L != 64 && L != 128)
        return fail(QLDPC_ERR_UNSUPPORTED, "code_create: lift size must be 16, 32, 64 or 128");

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
    code->shift.assign(host.shift, host.shift + kMaxSlots);
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) { delete code; return hip_fail(e, "hipGetDevice"); }
    e = hipSetDevice(device);
    if (e != hipSuccess) { delete code; return hip_fail(e, "hipSetDevice"); }
    e = hipMalloc(&code->dev, sizeof(DevCode));
    if (e != hipSuccess) {
        hipSetDevice(prev);
        delete code;
        return fail(QLDPC_ERR_OUT_OF_MEMORY, "code_create: hipMalloc failed");
    }
    e = hipMemcpy(code->dev, &host, sizeof(DevCode), hipMemcpyHostToDevice);
    hipSetDevice(prev);
    if (e != hipSuccess) {
        hipFree(code->dev);
        delete code;
        return hip_fail(e, "code_create: upload");
    }
    *out = code;
    return QLDPC_OK;
}

qldpc_status qldpc_code_destroy(qldpc_code code) {
    if (!code) return QLDPC_OK;
    if (code->dev) hipFree(code->dev);
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

qldpc_status qldpc_decode_batch(qldpc_code code, const qldpc_decode_params *p, int32_t batch,
                                const uint32_t *syn, const void *priors, uint32_t *err,
                                uint8_t *conv, uint8_t *iters, float *post, void *stream) {
    if (!code || !p) return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: null code or params");
    if (batch < 0) return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: negative batch");
    if (p->max_iters < 1 || p->max_iters > 255)
        return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: max_iters must be in [1, 255]");
    if (p->fmt != QLDPC_F32 && p->fmt != QLDPC_I8Q4) return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: bad format");
    if (p->sched != QLDPC_FLOOD && p->sched != QLDPC_LAYERED)
        return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: bad schedule");
    if (p->prior_mode != QLDPC_PRIOR_PER_SHOT && p->prior_mode != QLDPC_PRIOR_PER_BIT)
        return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: bad prior mode");
    if (!(p->alpha > 0.0f && p->alpha <= 1.0f)) return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: alpha must be in (0, 1]");
    if (batch == 0) return QLDPC_OK;
    if (!syn || !priors || !err || !conv) return fail(QLDPC_ERR_INVALID_ARG, "decode_batch: null buffer");
    DecodeArgs a{};
    a.code = code->dev;
    a.syn = syn;
    a.prior = priors;
    a.err = err;
    a.conv = conv;
    a.iters = iters;
    a.post = post;
    a.batch = batch;
    a.max_iters = p->max_iters;
    a.early_stop = p->early_stop ? 1 : 0;
    a.alpha = p->alpha;
    if (p->fmt == QLDPC_I8Q4) {
        int sh = 0;
        for (; sh <= 8; ++sh) {
            const float num = p->alpha * (float)(1 << sh);
            if (num == std::floor(num)) break;
        }
        if (sh > 8) return fail(QLDPC_ERR_UNSUPPORTED, "decode_batch: int8 needs alpha = num / 2^s, s <= 8");
        a.alpha_num = (int32_t)(p->alpha * (float)(1 << sh));
        a.alpha_shift = sh;
    }
    LaunchKey k{};
    k.which = code->which;
    k.L = code->L;
    k.fmt = p->fmt;
    k.sched = p->sched;
    k.per_bit = p->prior_mode == QLDPC_PRIOR_PER_BIT;
    k.post = post != nullptr;
    k.layout = p->layout == QLDPC_LAYOUT_AUTO ? QLDPC_LAYOUT_WAVE : p->layout;
    const hipError_t e = launch_decode(k, a, (hipStream_t)stream);
    if (e == hipErrorNotSupported)
        return fail(QLDPC_ERR_UNSUPPORTED, "decode_batch: no kernel for this format/schedule/layout/L");
    if (e != hipSuccess) return hip_fail(e, "decode_batch launch");
    return QLDPC_OK;
}

}  // extern "C"
