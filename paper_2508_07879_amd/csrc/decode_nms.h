// Neural min-sum: flooding min-sum (Section 2, Algorithm 1) whose check rule
// scales every edge by its own per-iteration weight w[k][e] instead of the
// single normalisation factor alpha.  FP32, T iterations, no early stop,
// per-shot priors.  Wavefront-per-shot mapping and LDS layout of the
// throughput decoder (decode_wave.h).
//
// Forward: writes every iteration's posterior Q^(k) and saves the inputs of
// every check pass, q^(k-1), to the workspace (one 120-slot LDS image per
// wave and iteration, stored lane-contiguous).
//
// Backward (reverse-mode derivative written out by hand), sweeping
// k = T .. 1 with g_q^(T) = 0:
//   variable side: g_r_e = G_n^(k) + sum over the other edges of n of g_q;
//   check side:    dL/dw_e += g_r_e * sgn_e * mag_e, and the only route from
//                  r_e back to q^(k-1) is the edge a that attains the excluded
//                  minimum: g_q_a += g_r_e * w_e * sgn_e * sg(q_a).
// Ties: the argmin is the lowest edge index (i1 = first index of min1; the
// edge paired with i1's own output is the first other index attaining
// min2).  Each wave accumulates its shots' weight gradients in its own
// partial slice (plain read-modify-write, no atomics); a reduction kernel
// sums the slices in a fixed order, so gradients are bit-reproducible.
#pragma once
#include "decode_wave.h"

namespace qldpc {

struct NmsArgs {
    const DevCode *code;
    const uint32_t *syn;     // [batch][syn_words]
    const float *prior;      // [batch]
    const float *w;          // [T][nnz], edge = CSR position (check-major, column order)
    float *post;             // forward: [T][batch][n]
    const float *gpost;      // backward: [T][batch][n]
    float *traj;             // [T][tiles][SLOTS * ROW]
    float *partial;          // [waves][T][SLOTS * ROW]
    float *grad_w;           // [T][nnz]
    int32_t batch;
    int32_t T;
    int32_t tiles;           // ceil(batch / shots per wave)
    int32_t waves;           // backward grid size (partial slices)
};


template <class S, int L>
__global__ __launch_bounds__(64) void k_nms_fwd(const NmsArgs a) {
    using namespace wave;
    using G = Geo<S, L>;
    constexpr int MB = S::MB, NB = S::NB, DC = S::DC, PPL = G::PPL, ROW = G::ROW, SLOTS = S::SLOTS;
    constexpr int NNZ = MB * L * DC;
    __shared__ __attribute__((aligned(16))) float msg[SLOTS * ROW];
    const int lane = threadIdx.x;
    const int g = lane / G::SEG, p = lane % G::SEG;
    const int tile = blockIdx.x;
    const long shot = (long)tile * G::SPW + g;
    const bool valid = shot < a.batch;
    const DevCode *__restrict__ code = a.code;

    uint32_t sb[PPL];
#pragma unroll
    for (int h = 0; h < PPL; ++h) {
        sb[h] = 0;
        if (valid)
#pragma unroll
            for (int R = 0; R < MB; ++R) {
                const int m = R * L + p + 64 * h;
                sb[h] |= ((a.syn[shot * G::SW + (m >> 5)] >> (m & 31)) & 1u) << R;
            }
    }
    const float gam = valid ? a.prior[shot] + 0.0f : 1.0f;
    static_for<0, NB>([&](auto Cc) {
        constexpr int C = decltype(Cc)::value;
        static_for<0, S::T.col_deg[C]>([&](auto Ii) {
            constexpr int i = decltype(Ii)::value;
            constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
            const uint32_t s = (uint32_t)code->shift[slot];
#pragma unroll
            for (int h = 0; h < PPL; ++h) msg[slot * ROW + vn_index<L>(lane, h, s)] = gam;
        });
    });
    for (int k = 0; k < a.T; ++k) {
        __builtin_amdgcn_wave_barrier();
        // save the check-node inputs q^(k)
        float *tr = a.traj + ((size_t)k * a.tiles + tile) * (SLOTS * ROW);
#pragma unroll 8
        for (int sl = 0; sl < SLOTS; ++sl)
#pragma unroll
            for (int h = 0; h < PPL; ++h) tr[sl * ROW + lane + 64 * h] = msg[sl * ROW + lane + 64 * h];
        // weighted check pass
#pragma unroll
        for (int R = 0; R < MB; ++R)
#pragma unroll
            for (int h = 0; h < PPL; ++h) {
                float v[DC], wj[DC];
#pragma unroll
                for (int j = 0; j < DC; ++j) v[j] = msg[(R * DC + j) * ROW + lane + 64 * h];
                load_weights<L, DC>(a.w, k, NNZ, R, p + 64 * h, wj);
                cn_f32_weighted<DC>(v, sb[h] << (31 - R), wj);
#pragma unroll
                for (int j = 0; j < DC; ++j) msg[(R * DC + j) * ROW + lane + 64 * h] = v[j];
            }
        __builtin_amdgcn_wave_barrier();
        // variable pass and posterior of iteration k + 1
        static_for<0, NB>([&](auto Cc) {
            constexpr int C = decltype(Cc)::value;
            constexpr int d = S::T.col_deg[C];
#pragma unroll
            for (int h = 0; h < PPL; ++h) {
                float r[d];
                int idx[d];
                static_for<0, d>([&](auto Ii) {
                    constexpr int i = decltype(Ii)::value;
                    constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                    idx[i] = slot * ROW + vn_index<L>(lane, h, (uint32_t)code->shift[slot]);
                    r[i] = msg[idx[i]];
                });
                float pre[d + 1];
                pre[0] = gam;
#pragma unroll
                for (int i = 0; i < d; ++i) pre[i + 1] = pre[i] + r[i];
#pragma unroll
                for (int i = 0; i < d; ++i) {
                    float q = pre[i];
#pragma unroll
                    for (int j = i + 1; j < d; ++j) q = q + r[j];
                    msg[idx[i]] = q;
                }
                if (valid) a.post[((size_t)k * a.batch + shot) * G::N + C * L + p + 64 * h] = pre[d];
            }
        });
    }
}

template <class S, int L>
__global__ __launch_bounds__(64) void k_nms_bwd(const NmsArgs a) {
    using namespace wave;
    using G = Geo<S, L>;
    constexpr int MB = S::MB, NB = S::NB, DC = S::DC, PPL = G::PPL, ROW = G::ROW, SLOTS = S::SLOTS;
    constexpr int NNZ = MB * L * DC;
    __shared__ __attribute__((aligned(16))) float gm[SLOTS * ROW];   // g_q / g_r per edge
    const int lane = threadIdx.x;
    const int g = lane / G::SEG, p = lane % G::SEG;
    const DevCode *__restrict__ code = a.code;
    const int wv = blockIdx.x;
    float *part = a.partial + (size_t)wv * a.T * (SLOTS * ROW);

    for (int tile = wv; tile < a.tiles; tile += a.waves) {
        const bool first = tile == wv;
        const long shot = (long)tile * G::SPW + g;
        const bool valid = shot < a.batch;
        uint32_t sb[PPL];
#pragma unroll
        for (int h = 0; h < PPL; ++h) {
            sb[h] = 0;
            if (valid)
#pragma unroll
                for (int R = 0; R < MB; ++R) {
                    const int m = R * L + p + 64 * h;
                    sb[h] |= ((a.syn[shot * G::SW + (m >> 5)] >> (m & 31)) & 1u) << R;
                }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll 8
        for (int sl = 0; sl < SLOTS; ++sl)
#pragma unroll
            for (int h = 0; h < PPL; ++h) gm[sl * ROW + lane + 64 * h] = 0.0f;   // g_q^(T) = 0
        for (int k = a.T - 1; k >= 0; --k) {
            __builtin_amdgcn_wave_barrier();
            // variable side: g_r = G + excluded sum of g_q, in place
            static_for<0, NB>([&](auto Cc) {
                constexpr int C = decltype(Cc)::value;
                constexpr int d = S::T.col_deg[C];
#pragma unroll
                for (int h = 0; h < PPL; ++h) {
                    float x[d];
                    int idx[d];
                    static_for<0, d>([&](auto Ii) {
                        constexpr int i = decltype(Ii)::value;
                        constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                        idx[i] = slot * ROW + vn_index<L>(lane, h, (uint32_t)code->shift[slot]);
                        x[i] = gm[idx[i]];
                    });
                    const float Gn = valid ? a.gpost[((size_t)k * a.batch + shot) * G::N + C * L + p + 64 * h] : 0.0f;
                    float pre[d + 1];
                    pre[0] = Gn;
#pragma unroll
                    for (int i = 0; i < d; ++i) pre[i + 1] = pre[i] + x[i];
#pragma unroll
                    for (int i = 0; i < d; ++i) {
                        float s = pre[i];
#pragma unroll
                        for (int j = i + 1; j < d; ++j) s = s + x[j];
                        gm[idx[i]] = s;
                    }
                }
            });
            __builtin_amdgcn_wave_barrier();
            // check side: weight gradients and g_q^(k)
            const float *tr = a.traj + ((size_t)k * a.tiles + tile) * (SLOTS * ROW);
            float *pk = part + (size_t)k * (SLOTS * ROW);
#pragma unroll
            for (int R = 0; R < MB; ++R)
#pragma unroll
                for (int h = 0; h < PPL; ++h) {
                    float q[DC], gr[DC], wj[DC];
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        q[j] = tr[(R * DC + j) * ROW + lane + 64 * h];
                        gr[j] = gm[(R * DC + j) * ROW + lane + 64 * h];
                    }
                    load_weights<L, DC>(a.w, k, NNZ, R, p + 64 * h, wj);
                    float m1 = INFINITY, m2 = INFINITY;
                    int i1 = 0, i2 = 0;
                    uint32_t P = sb[h] << (31 - R);
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        const float av = fabsf(q[j]);
                        if (av < m1) {
                            m2 = m1;
                            i2 = i1;
                            m1 = av;
                            i1 = j;
                        } else if (av < m2) {
                            m2 = av;
                            i2 = j;
                        }
                        P ^= fbits(q[j]);
                    }
                    float c[DC];
                    float acc_i1 = 0.0f;
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        const float sgn = ((P ^ fbits(q[j])) & 0x80000000u) ? -1.0f : 1.0f;
                        const float mag = (j == i1) ? m2 : m1;
                        const float dw = gr[j] * sgn * mag;
                        float *dst = pk + (R * DC + j) * ROW + lane + 64 * h;
                        *dst = first ? dw : (*dst + dw);
                        c[j] = gr[j] * wj[j] * sgn;
                        if (j != i1) acc_i1 = acc_i1 + c[j];
                    }
                    float c_i1 = 0.0f;
#pragma unroll
                    for (int j = 0; j < DC; ++j) c_i1 = (j == i1) ? c[j] : c_i1;
                    float sq1 = 1.0f, sq2 = 1.0f;
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        const float sj = q[j] < 0.0f ? -1.0f : 1.0f;
                        sq1 = (j == i1) ? sj : sq1;
                        sq2 = (j == i2) ? sj : sq2;
                    }
#pragma unroll
                    for (int j = 0; j < DC; ++j) {
                        float o = 0.0f;
                        if (j == i1) o = acc_i1 * sq1;
                        if (j == i2) o = c_i1 * sq2;
                        gm[(R * DC + j) * ROW + lane + 64 * h] = o;
                    }
                }
        }
    }
}

// grad_w[k][e] = sum over waves (in order) and over the shot segments of a
// wave (in order) of the partial slices.
template <class S, int L>
__global__ __launch_bounds__(256) void k_nms_reduce(const NmsArgs a) {
    using G = Geo<S, L>;
    constexpr int DC = S::DC, ROW = G::ROW, SLOTS = S::SLOTS;
    constexpr int NNZ = S::MB * L * DC;
    // one thread per (k, slot, circulant row) with rows innermost
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)a.T * SLOTS * L;
    if (i >= total) return;
    const int pos = (int)(i % L);
    const int sl = (int)((i / L) % SLOTS);
    const int k = (int)(i / ((long)L * SLOTS));
    float acc = 0.0f;
    for (int wv = 0; wv < a.waves; ++wv) {
        const float *pk = a.partial + ((size_t)wv * a.T + k) * (SLOTS * ROW) + sl * ROW;
        if constexpr (L <= 64) {
#pragma unroll
            for (int g = 0; g < G::SPW; ++g) acc += pk[g * L + pos];
        } else {
            acc += pk[pos];
        }
    }
    const int R = sl / DC, j = sl % DC;
    a.grad_w[(size_t)k * NNZ + (size_t)(R * L + pos) * DC + j] = acc;
}

}  // namespace qldpc
