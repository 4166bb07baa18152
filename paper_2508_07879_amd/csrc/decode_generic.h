// Min-sum decoder for a parity-check matrix given only as edge lists (no
// quasi-cyclic lift): Section 2, Algorithm 1, flooding schedule, over the
// CSR form of H (check-node pass) and its CSC form (variable-node pass).
//
// Mapping.  One wavefront decodes one shot.  Lane l visits checks l, l + 64,
// ... in the check pass and variables l, l + 64, ... in the variable pass.
// Edge messages live in LDS, slot-major: the message on the j-th edge of
// check r (CSR order) is msg[j * m + r], so in the check pass consecutive
// lanes touch consecutive words (no bank conflicts whatever the degrees).
// The variable pass reaches its edges through the table vn_slot, which holds
// j * m + r for the k-th edge of variable v in increasing check order.
// Packed decisions and the shot's syndrome are staged in LDS as well; the
// tables stay in device memory, read through the caches by every wave.
//
// Numerics are those of the lifted kernels: FP32 excluded sums left to right
// from gamma_v in increasing check index, alpha * min rounded once, no
// contraction, priors canonicalised with + 0.0f; integer formats (int8 with
// Q4 priors, int16 with Q8 priors) saturate q to [-qmax, qmax] and compute
// r = sign * ((num * min) >> sh) with exact integer sums.
#pragma once
#include <stdint.h>

#include "decode_generic_api.h"
#include "decode_wave.h"

namespace qldpc {

namespace gen {

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Excluded sums of one variable of degree d whose incoming messages sit at
// LDS indices slot[0 .. d-1] (increasing check order), written back in
// place; returns the a-posteriori sum.  FP32: q_i = (...((gamma + r_0) + ...
// + r_{i-1}) + r_{i+1}) + ... + r_{d-1}, i.e. the prefix before i continued
// over the edges after i.
template <int FMT>
__device__ __forceinline__ float vn_f32(float *msg, const int32_t *__restrict__ slots, int d, float gam) {
    constexpr int U = 8;   // degrees up to U run from registers
    if (d <= U) {
        int sl[U];
        float r[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            sl[k] = k < d ? slots[k] : 0;
            r[k] = k < d ? msg[sl[k]] : 0.0f;
        }
        float pre = gam;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            if (i < d) {
                float q = pre;
#pragma unroll
                for (int j = i + 1; j < U; ++j)
                    if (j < d) q = q + r[j];
                msg[sl[i]] = q;
                pre = pre + r[i];
            }
        }
        return pre;
    }
    float pre = gam;
    for (int i = 0; i < d; ++i) {
        const int si = slots[i];
        const float ri = msg[si];
        float q = pre;
        for (int j = i + 1; j < d; ++j) q = q + msg[slots[j]];
        msg[si] = q;
        pre = pre + ri;
    }
    return pre;
}

}  // namespace gen

// One wavefront per shot; grid = batch; dynamic LDS = gen_lds_bytes(...).
template <int FMT, bool PER_BIT, bool POST>
__global__ __launch_bounds__(64) void k_gen(const GenCode g, const DecodeArgs a) {
    using msg_t = typename Fmt<FMT>::msg_t;
    using prior_t = typename Fmt<FMT>::prior_t;
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int m = g.m, n = g.n;
    const int SW = (m + 31) / 32, EW = (n + 31) / 32;
    msg_t *msg = reinterpret_cast<msg_t *>(lds);
    uint32_t *ebits = reinterpret_cast<uint32_t *>(lds + (((size_t)g.max_dc * m * sizeof(msg_t) + 15) & ~size_t(15)));
    uint32_t *sbits = ebits + EW;

    const long shot = xcd_wave_index(blockIdx.x, gridDim.x);
    if (shot >= a.batch) return;                       // wave-uniform
    if (a.only && a.only[shot] == 0) return;
    const int lane = threadIdx.x & 63;
    const uint32_t *syn = a.syn + shot * SW;
    for (int w = lane; w < SW; w += 64) sbits[w] = syn[w];
    const prior_t *pr = static_cast<const prior_t *>(a.prior);
    auto gamma_of = [&](int v) -> float {
        float x = PER_BIT ? (float)pr[shot * n + v] : (float)pr[shot];
        if constexpr (FMT == 0) x = x + 0.0f;
        return x;
    };
    // q^(0) = gamma on every edge
    for (int v = lane; v < n; v += 64) {
        const msg_t gv = (msg_t)gamma_of(v);
        for (int k = g.col_ptr[v]; k < g.col_ptr[v + 1]; ++k) msg[g.vn_slot[k]] = gv;
    }
    gen::wave_sync_lds();

    const int vrounds = (n + 63) / 64;
    for (int k = 1; k <= a.max_iters; ++k) {
        // ---------------- check-node pass (CSR rows) ----------------------
        for (int r = lane; r < m; r += 64) {
            const int d = g.row_ptr[r + 1] - g.row_ptr[r];
            const uint32_t s = (sbits[r >> 5] >> (r & 31)) & 1u;
            if constexpr (FMT == 0) {
                float m1 = INFINITY, m2 = INFINITY;
                uint32_t P = s << 31;
                for (int j = 0; j < d; ++j) {
                    const float x = msg[j * m + r];
                    const float ax = fabsf(x);
                    m2 = __builtin_amdgcn_fmed3f(m1, m2, ax);
                    m1 = fminf(m1, ax);
                    P ^= __float_as_uint(x);
                }
                const float A1 = a.alpha * m1, A2 = a.alpha * m2;
                for (int j = 0; j < d; ++j) {
                    const float x = msg[j * m + r];
                    const float mag = (fabsf(x) == m1) ? A2 : A1;
                    msg[j * m + r] = __uint_as_float(__float_as_uint(mag) | ((P ^ __float_as_uint(x)) & 0x80000000u));
                }
            } else {
                int m1 = 1 << 30, m2 = 1 << 30;
                uint32_t P = s << 31;
                for (int j = 0; j < d; ++j) {
                    const int x = (int)msg[j * m + r];
                    const int ax = x < 0 ? -x : x;
                    m2 = max(m1, min(m2, ax));
                    m1 = min(m1, ax);
                    P ^= (uint32_t)x;
                }
                const int A1 = (a.alpha_num * m1) >> a.alpha_shift;
                const int A2 = (a.alpha_num * m2) >> a.alpha_shift;
                for (int j = 0; j < d; ++j) {
                    const int x = (int)msg[j * m + r];
                    const int ax = x < 0 ? -x : x;
                    const int mag = ax == m1 ? A2 : A1;
                    msg[j * m + r] = (msg_t)(((int)(P ^ (uint32_t)x) < 0) ? -mag : mag);
                }
            }
        }
        gen::wave_sync_lds();
        // ---------------- variable-node pass (CSC columns) -----------------
        for (int i = 0; i < vrounds; ++i) {
            const int v = i * 64 + lane;
            bool e = false;
            if (v < n) {
                const int base = g.col_ptr[v], d = g.col_ptr[v + 1] - base;
                float Q;
                if constexpr (FMT == 0) {
                    Q = gen::vn_f32<FMT>(reinterpret_cast<float *>(msg), g.vn_slot + base, d, gamma_of(v));
                } else {
                    int sum = (int)gamma_of(v);
                    for (int t = 0; t < d; ++t) sum += (int)msg[g.vn_slot[base + t]];
                    for (int t = 0; t < d; ++t) {
                        const int sl = g.vn_slot[base + t];
                        msg[sl] = (msg_t)wave::sat<FMT>(sum - (int)msg[sl]);
                    }
                    Q = (float)sum;
                }
                e = Q < 0.0f;
                if constexpr (POST) a.post[shot * n + v] = FMT == 0 ? Q : Q * Fmt<FMT>::post_scale;
            }
            const uint64_t mask = __ballot(e);
            if (lane < 2 && 2 * i + lane < EW) ebits[2 * i + lane] = (uint32_t)(mask >> (32 * lane));
        }
        gen::wave_sync_lds();
        // ---------------- syndrome test and stopping rule ------------------
        bool unsat = false;
        for (int r = lane; r < m; r += 64) {
            uint32_t par = (sbits[r >> 5] >> (r & 31)) & 1u;
            for (int f = g.row_ptr[r]; f < g.row_ptr[r + 1]; ++f) {
                const int c = g.col_idx[f];
                par ^= (ebits[c >> 5] >> (c & 31)) & 1u;
            }
            unsat = unsat || par != 0;
        }
        const bool conv = __ballot(unsat) == 0;
        if ((a.early_stop && conv) || k == a.max_iters) {
            uint32_t *err = a.err + shot * EW;
            for (int w = lane; w < EW; w += 64) err[w] = ebits[w];
            if (lane == 0) {
                a.conv[shot] = conv ? 1 : 0;
                if (a.iters) a.iters[shot] = (uint8_t)k;
            }
            return;
        }
    }
}

}  // namespace qldpc
