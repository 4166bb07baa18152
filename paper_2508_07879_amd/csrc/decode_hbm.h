// Workgroup-per-shot min-sum decoder with the edge messages in device memory
// (HBM), for lifted codes whose messages do not fit on chip (L = 256, 512;
// any L >= 64 works).  Flooding schedule (Section 2, Algorithm 1).
//
// One workgroup of NW wavefronts decodes one shot.  The shot's messages live
// in a caller-provided workspace, slot-major: msg[(R*8 + j)*L + t] is the
// message on the edge of check (R, t) in slot j, so a check pass touches 64
// consecutive entries per wave instruction and a variable pass a rotated
// row (at most two runs).  A work item is one 64-row slice of a block row
// (check pass) or of a block column (variable pass), looped at run time
// (the pattern tables are read from constant memory): the kernel is bound by
// HBM traffic, 4 E b bytes per iteration, not by instruction issue, and
// its code size stays independent of L.
//
// Per iteration k: check pass of k and, per block row, the syndrome test of
// the decisions of k-1 (multi-word rotations of 64-bit ballots held in LDS,
// on the scalar unit); barrier; all checks satisfied -> emit k-1 and stop;
// variable pass, a posteriori, decisions; barrier.  After the last
// iteration one more test decides the flag.  Posteriors, when requested,
// are written every iteration (the last write is the result).
#pragma once
#include "decode_wave.h"

namespace qldpc {

template <class S, int L, int NW>
struct HbmLds {
    static constexpr int PPL = L / 64;
    static constexpr size_t e_off = 0;                                  // uint64 [NB][PPL]
    static constexpr size_t f_off = e_off + (size_t)S::NB * PPL * 8;    // uint32 flags[2]
    static constexpr size_t s_off = f_off + 16;                         // uint32 syndrome words
    static constexpr size_t bytes = s_off + (((size_t)S::MB * L + 31) / 32) * 4;
};

// Word w of the L-bit vector e (PPL 64-bit words, in LDS) rotated right by
// s: bit t of the result is bit (t + s) mod L of e.
template <int L>
__device__ __forceinline__ uint64_t rot_word(const uint64_t *e, uint32_t s, int w) {
    constexpr int PPL = L / 64;
    const uint32_t b = 64u * (uint32_t)w + s;
    const int q = (int)(b / 64u) % PPL;
    const uint32_t r = b % 64u;
    const uint64_t w0 = wave::uniform64(e[q]);
    if (r == 0) return w0;
    const uint64_t w1 = wave::uniform64(e[(q + 1) % PPL]);
    return (w0 >> r) | (w1 << (64u - r));
}

// Decodes shot `shot` of the code whose shift table is `code_table`
// (syndrome words at syn, error words to err, flags and priors indexed by
// shot) with the whole workgroup, messages at msg.  a.code is not used: the
// mixed-code path passes each shot's own table.  Every thread of the
// workgroup must call it; `lds` holds HbmLds<S, L, NW>::bytes.
template <class S, int L, int FMT, int NW, bool PER_BIT, bool POST>
__device__ __forceinline__ void hbm_decode(const DecodeArgs &a, const DevCode *code_table, const long shot,
                                           const uint32_t *syn, uint32_t *err, typename Fmt<FMT>::msg_t *msg,
                                           unsigned char *lds) {
    using namespace wave;
    static_assert(L >= 64 && L % 64 == 0, "HBM layout: L a multiple of 64");
    using Lay = HbmLds<S, L, NW>;
    using msg_t = typename Fmt<FMT>::msg_t;
    using prior_t = typename Fmt<FMT>::prior_t;
    using acc_t = typename std::conditional<FMT == 0, float, int>::type;
    constexpr int MB = S::MB, NB = S::NB, DC = S::DC, PPL = L / 64;
    constexpr int N = NB * L, SW = (MB * L + 31) / 32, EW = (NB * L + 31) / 32;
    constexpr int CN_ITEMS = MB * PPL, VN_ITEMS = NB * PPL;

    uint64_t *emask = reinterpret_cast<uint64_t *>(lds + Lay::e_off);
    uint32_t *flag = reinterpret_cast<uint32_t *>(lds + Lay::f_off);
    uint32_t *synw = reinterpret_cast<uint32_t *>(lds + Lay::s_off);

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const CodePtr code = const_code(code_table);
    const prior_t *prior = static_cast<const prior_t *>(a.prior);

    for (int w = threadIdx.x; w < SW; w += 64 * NW) synw[w] = syn[w];
    acc_t gshot = 0;
    if constexpr (!PER_BIT) {
        gshot = (acc_t)prior[shot];
        if constexpr (FMT == 0) gshot = gshot + 0.0f;   // no -0.0 in any message
    }
    auto gamma_at = [&](int C, int h) -> acc_t {
        if constexpr (PER_BIT) {
            acc_t v = (acc_t)prior[shot * N + C * L + 64 * h + lane];
            if constexpr (FMT == 0) v = v + 0.0f;
            return v;
        } else {
            return gshot;
        }
    };
    // position in a slot row of the entry that variable (C, 64 h + lane) reaches through shift s
    auto vn_pos = [&](int h, uint32_t s) -> int { return (int)(((uint32_t)(64 * h + lane) - s) & (uint32_t)(L - 1)); };

    // q^(0) = gamma on every edge
    for (int it = wv; it < VN_ITEMS; it += NW) {
        const int C = it / PPL, h = it % PPL;
        const acc_t g = gamma_at(C, h);
        for (int i = 0; i < S::T.col_deg[C]; ++i) {
            const int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
            msg[slot * L + vn_pos(h, (uint32_t)code->shift[slot])] = (msg_t)g;
        }
    }
    if (threadIdx.x == 0) {
        flag[0] = 0;
        flag[1] = 0;
    }
    __syncthreads();

    auto syn_bit = [&](int R, int h) -> uint32_t {
        const int m = R * L + 64 * h + lane;
        return (synw[m >> 5] >> (m & 31)) & 1u;
    };
    auto emit = [&](int k, bool conv) {
        for (int w = threadIdx.x; w < EW; w += 64 * NW) {
            const uint64_t m = emask[(w * 32) / 64];
            err[w] = (uint32_t)(m >> ((w * 32) % 64));
        }
        if (threadIdx.x == 0) {
            a.conv[shot] = conv ? 1 : 0;
            if (a.iters) a.iters[shot] = (uint8_t)k;
        }
    };
    // syndrome test of the decisions in emask; raises flag[par] on a violation
    auto test_rows = [&](int par) {
        for (int it = wv; it < CN_ITEMS; it += NW) {
            const int R = it / PPL, h = it % PPL;
            uint64_t c = ballot(syn_bit(R, h) != 0);
            for (int j = 0; j < DC; ++j) {
                const int C = S::T.slot_bc[R][j];
                c ^= rot_word<L>(emask + C * PPL, (uint32_t)code->shift[R * DC + j], h);
            }
            if (c != 0 && lane == 0) atomicOr(&flag[par], 1u);
        }
    };

    int k = 1;
    for (; k <= a.max_iters; ++k) {
        // ---- check pass of iteration k, test of iteration k-1 --------------
        for (int it = wv; it < CN_ITEMS; it += NW) {
            const int R = it / PPL, h = it % PPL;
            const uint32_t P = syn_bit(R, h) << 31;
            msg_t *row = msg + (R * DC) * L + 64 * h + lane;
            if constexpr (FMT == 0) {
                float v[DC];
#pragma unroll
                for (int j = 0; j < DC; ++j) v[j] = row[j * L];
                cn_f32<DC>(v, P, a.alpha);
#pragma unroll
                for (int j = 0; j < DC; ++j) row[j * L] = v[j];
            } else {
                int v[DC];
#pragma unroll
                for (int j = 0; j < DC; ++j) v[j] = row[j * L];
                cn_fx<DC>(v, P, a.alpha_num, a.alpha_shift);
#pragma unroll
                for (int j = 0; j < DC; ++j) row[j * L] = (msg_t)v[j];
            }
        }
        if (k > 1 && a.early_stop) test_rows(k & 1);
        __syncthreads();
        if (k > 1 && a.early_stop && __builtin_amdgcn_readfirstlane(flag[k & 1]) == 0) {   // uniform
            emit(k - 1, true);
            return;
        }
        // ---- variable pass, a posteriori, decisions ------------------------
        for (int it = wv; it < VN_ITEMS; it += NW) {
            const int C = it / PPL, h = it % PPL;
            const int d = S::T.col_deg[C];
            acc_t r[kMaxDv];
            int idx[kMaxDv];
#pragma unroll
            for (int i = 0; i < kMaxDv; ++i) {
                if (i < d) {
                    const int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                    idx[i] = slot * L + vn_pos(h, (uint32_t)code->shift[slot]);
                    r[i] = (acc_t)msg[idx[i]];
                }
            }
            acc_t Q;
            if constexpr (FMT == 0) {
                // prefix sums from gamma in increasing check order; the
                // excluded sum of edge i continues the prefix before i
                float pre[kMaxDv + 1];
                pre[0] = gamma_at(C, h);
#pragma unroll
                for (int i = 0; i < kMaxDv; ++i)
                    if (i < d) pre[i + 1] = pre[i] + r[i];
#pragma unroll
                for (int i = 0; i < kMaxDv; ++i) {
                    if (i < d) {
                        float q = pre[i];
#pragma unroll
                        for (int j = i + 1; j < kMaxDv; ++j)
                            if (j < d) q = q + r[j];
                        msg[idx[i]] = q;
                    }
                }
                Q = pre[d];
            } else {
                int sum = gamma_at(C, h);
#pragma unroll
                for (int i = 0; i < kMaxDv; ++i)
                    if (i < d) sum += r[i];
#pragma unroll
                for (int i = 0; i < kMaxDv; ++i)
                    if (i < d) msg[idx[i]] = (msg_t)sat<FMT>(sum - r[i]);
                Q = sum;
            }
            if constexpr (POST) {
                float qv;
                if constexpr (FMT == 0) qv = Q;
                else qv = (float)Q * Fmt<FMT>::post_scale;
                a.post[shot * N + C * L + 64 * h + lane] = qv;
            }
            const uint64_t m = ballot(Q < (acc_t)0);
            if (lane == 0) emask[C * PPL + h] = m;
        }
        if (threadIdx.x == 0) flag[(k + 1) & 1] = 0;
        __syncthreads();
    }
    // after the last iteration: one more test decides the flag
    --k;
    test_rows((k + 1) & 1);
    __syncthreads();
    emit(k, __builtin_amdgcn_readfirstlane(flag[(k + 1) & 1]) == 0);
}

template <class S, int L, int FMT, int NW, bool PER_BIT, bool POST>
__global__ __launch_bounds__(64 * NW) void k_hbm(const DecodeArgs a, void *workspace) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[HbmLds<S, L, NW>::bytes];
    constexpr int SW = (S::MB * L + 31) / 32, EW = (S::NB * L + 31) / 32;
    const long shot = blockIdx.x;
    if (a.only && a.only[shot] == 0) return;   // uniform over the workgroup
    using msg_t = typename Fmt<FMT>::msg_t;
    msg_t *msg = static_cast<msg_t *>(workspace) + shot * (long)(S::SLOTS * L);
    hbm_decode<S, L, FMT, NW, PER_BIT, POST>(a, a.code, shot, a.syn + shot * SW, a.err + shot * EW, msg, lds);
}

template <class S, int L, int FMT, int NW>
hipError_t launch_hbm(const LaunchKey &k, const DecodeArgs &a, void *ws, hipStream_t st) {
    const dim3 grid((unsigned)a.batch), block(64 * NW);
    if (k.per_bit) {
        if (k.post) hipLaunchKernelGGL((k_hbm<S, L, FMT, NW, true, true>), grid, block, 0, st, a, ws);
        else hipLaunchKernelGGL((k_hbm<S, L, FMT, NW, true, false>), grid, block, 0, st, a, ws);
    } else {
        if (k.post) hipLaunchKernelGGL((k_hbm<S, L, FMT, NW, false, true>), grid, block, 0, st, a, ws);
        else hipLaunchKernelGGL((k_hbm<S, L, FMT, NW, false, false>), grid, block, 0, st, a, ws);
    }
    return hipGetLastError();
}

}  // namespace qldpc
