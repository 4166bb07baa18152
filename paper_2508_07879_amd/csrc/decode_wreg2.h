// Register-resident decoder for the lift sizes L = 128, 256, 512: one
// workgroup of W = L / 64 wavefronts per shot, flooding schedule (Section 2,
// Algorithm 1).
//
// Mapping.  Wave w, lane t owns row r = 64 w + t of every L x L circulant:
// check (R, r) of each block row, with the 8 messages of its edges in
// registers (120 per lane, as in the L = 64 register decoder), and variable
// (C, r) of each block column.  The check pass works on registers only.  The
// variable pass needs the messages of checks (R, r - s mod L), which mostly
// live in other waves, so it goes through LDS, a batch of block columns at a
// time:
//   1. every lane stores its messages of the batch's edge slots at its own
//      row of an L-entry slot row;
//   2. barrier; every lane reads the messages of its variable at rows
//      r - s, forms the excluded sums in the oracle's order and writes each
//      new message back to the row it came from (same address); it also
//      XORs its decision e_(C, r), at bit R, into a per-row word of the
//      check it came from (an LDS atomic on the same row);
//   3. barrier; every lane reads its own rows back into its registers.
// A lane only ever writes or reads its own rows outside step 2, and step 2
// is fenced by the two barriers, so one buffer serves every batch.  All
// accesses are to consecutive rows or to the same rows rotated by the shift:
// no bank conflicts.  After the last batch, the word of row r, XOR the
// syndrome bits, is the syndrome test of the lane's 15 checks; the shot has
// converged when no wave found a violated check (flags in LDS, one more
// barrier per iteration).
//
// Numerics are those of the other layouts: FP32 excluded sums left to right
// from gamma in increasing check order, fl(alpha * min) once, no contraction;
// the integer formats run as exact integer values on FP32 lanes (cn_fxf,
// satf), as in the L <= 64 register decoder.
#pragma once
#include "decode_wave.h"

namespace qldpc {

namespace wreg2 {

// LDS views (address space 3), so that computed offsets stay 32-bit LDS
// addresses instead of generic pointers.
typedef __attribute__((address_space(3))) unsigned char lds_u8;
typedef __attribute__((address_space(3))) float lds_f32;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Block columns per LDS exchange batch.  L = 128, FP32, 3 x 32768 shots:
// 2, 4, 8, 12 columns ran 12.53, 12.79, 12.89, 12.91 M syndromes/s.  At
// L = 512 a batch of 4 keeps the exchange buffer at 30 KB.
template <int L>
constexpr int vb_of() { return L >= 512 ? 4 : 8; }

// Edge slots of the columns of batch B: their count and, per column, the
// index of its first slot inside the batch.
template <class S, int VB>
struct Batches {
    static constexpr int NBATCH = (S::NB + VB - 1) / VB;
    int count[NBATCH];
    int first[S::NB];
    int max_count;
};

template <class S, int VB>
constexpr Batches<S, VB> make_batches() {
    Batches<S, VB> b{};
    b.max_count = 0;
    for (int B = 0; B < Batches<S, VB>::NBATCH; ++B) {
        int n = 0;
        for (int C = B * VB; C < S::NB && C < (B + 1) * VB; ++C) {
            b.first[C] = n;
            n += S::T.col_deg[C];
        }
        b.count[B] = n;
        b.max_count = n > b.max_count ? n : b.max_count;
    }
    return b;
}

template <class S, int L>
struct BatchesOf {
    static constexpr int VB = vb_of<L>();
    static constexpr Batches<S, VB> V = make_batches<S, VB>();
};

template <class S, int FMT, int L>
struct Lds {
    static constexpr int W = L / 64;
    static constexpr int XS = BatchesOf<S, L>::V.max_count;
    float xq[XS][L];              // per slot of a batch: message row
    // Per circulant row: bit R = XOR of the decisions of the variables that
    // check (R, row) meets, accumulated by the variable pass with LDS atomics.
    uint32_t eacc[L];
    uint32_t unsat[2][W];         // per iteration parity, per wave: a violated check
};

}  // namespace wreg2

// Decodes one shot with the L / 64 waves of the calling workgroup (every wave
// must call it with the same, workgroup-uniform arguments): `syn` and `err`
// point at the shot's syndrome and error words, priors, flags and the
// a-posteriori output are indexed by `shot`.  Leaves with every wave at the
// same iteration; the caller fences LDS before reusing `sh`.
template <class S, int FMT, bool PER_BIT, bool POST, int L>
__device__ __forceinline__ void wreg2_decode(const DecodeArgs &a, const DevCode *code, const long shot,
                                             const uint32_t *syn, uint32_t *err_shot, wreg2::Lds<S, FMT, L> &sh) {
    using namespace wave;
    using B = wreg2::BatchesOf<S, L>;
    using prior_t = typename Fmt<FMT>::prior_t;
    static_assert(L == 128 || L == 256 || L == 512, "one wave per 64 circulant rows");
    constexpr int MB = S::MB, NB = S::NB, DC = S::DC, N = NB * L, W = L / 64, VB = B::VB;
    constexpr int NBATCH = B::V.NBATCH;

    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = threadIdx.x & 63;
    const uint32_t r = (uint32_t)(64 * w + t);                     // this lane's circulant row
    const uint32_t r4 = r << 2;
    const CodePtr cpb0 = const_code(code);
    CodePtr cpb = cpb0;
    auto reload_table = [&]() {
        uint64_t v = (uint64_t)code;
        asm volatile("" : "+s"(v));
        cpb = (CodePtr)v;
    };

    // syndrome bits of this lane's checks: bit R = s of check R * L + r
    uint32_t sb = 0;
#pragma unroll
    for (int R = 0; R < MB; ++R) {
        const uint32_t m = (uint32_t)R * L + r;
        sb |= ((syn[m >> 5] >> (m & 31)) & 1u) << R;
    }
    // priors (FP32 canonicalised so that no message is -0.0)
    const prior_t *pr = static_cast<const prior_t *>(a.prior);
    auto prior_at = [&](int C, uint32_t row) -> float {
        float v = PER_BIT ? (float)pr[shot * N + C * L + row] : (float)pr[shot];
        if constexpr (FMT == 0) v = v + 0.0f;
        return v;
    };
    float gam[PER_BIT ? NB : 1];
    if constexpr (PER_BIT) {
#pragma unroll
        for (int C = 0; C < NB; ++C) gam[C] = prior_at(C, r);
    } else {
        gam[0] = prior_at(0, r);
    }
    auto gamma_of = [&](int C) -> float { return PER_BIT ? gam[C] : gam[0]; };

    // q^(0) = gamma: the check at row r of slot (R, j) meets variable
    // (C, r + s mod L)
    float m[S::SLOTS];
    static_for<0, MB>([&](auto Rc) {
        constexpr int R = decltype(Rc)::value;
        static_for<0, DC>([&](auto Jc) {
            constexpr int j = decltype(Jc)::value;
            constexpr int C = S::T.slot_bc[R][j];
            if constexpr (PER_BIT) {
                const uint32_t s = (uint32_t)cpb0->shift[R * DC + j];
                m[R * DC + j] = prior_at(C, (r + s) & (L - 1));
            } else {
                m[R * DC + j] = gamma_of(C);
            }
        });
    });

    float Qr[POST ? NB : 1];
    for (int k = 1; k <= a.max_iters; ++k) {
        // ---------------- check-node pass: registers only -------------------
#pragma unroll
        for (int R = 0; R < MB; ++R) {
            const uint32_t P = sb << (31 - R);
            float v[DC];
#pragma unroll
            for (int j = 0; j < DC; ++j) v[j] = m[R * DC + j];
            if constexpr (FMT == 0) cn_f32<DC>(v, P, a.alpha);
            else cn_fxf<DC>(v, P, a.alpha);
#pragma unroll
            for (int j = 0; j < DC; ++j) m[R * DC + j] = v[j];
        }
        uint64_t eb = 0;        // bit C: e of variable (C, r)
        sh.eacc[r] = 0;         // this lane's row; the first batch's barrier orders it
        // ---------------- variable pass, a batch of columns at a time -------
        static_for<0, NBATCH>([&](auto Bc) {
            constexpr int b = decltype(Bc)::value;
            constexpr int C0 = b * VB;
            constexpr int C1 = (C0 + VB < NB) ? C0 + VB : NB;
            // 1. own messages of the batch's slots, at this lane's row
            static_for<C0, C1>([&](auto Cc) {
                constexpr int C = decltype(Cc)::value;
                static_for<0, S::T.col_deg[C]>([&](auto Ic) {
                    constexpr int i = decltype(Ic)::value;
                    constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                    sh.xq[B::V.first[C] + i][r] = m[slot];
                });
            });
            __syncthreads();
            // 2. the variables of this lane: messages from rows r - s, new
            //    messages and this variable's decision back to those rows
            reload_table();
            static_for<C0, C1>([&](auto Cc) {
                constexpr int C = decltype(Cc)::value;
                constexpr int d = S::T.col_deg[C];
                float rr[d];
                uint32_t ad[d];
                static_for<0, d>([&](auto Ic) {
                    constexpr int i = decltype(Ic)::value;
                    // byte offset of row (r - s) mod L: (4r + 4c) mod 4L, c = (L - s) mod L
                    const uint32_t c4 = (uint32_t)cpb->colrot[C][i].c4;
                    ad[i] = (r4 + c4) & (uint32_t)(4 * L - 4);
                    wreg2::lds_u8 *row = (wreg2::lds_u8 *)&sh.xq[B::V.first[C] + i][0];
                    rr[i] = *(wreg2::lds_f32 *)(row + ad[i]);
                });
                float qv[d], Q;
                if constexpr (FMT == 0) {
                    float pre[d + 1];
                    pre[0] = gamma_of(C);
#pragma unroll
                    for (int i = 0; i < d; ++i) pre[i + 1] = pre[i] + rr[i];
#pragma unroll
                    for (int i = 0; i < d; ++i) {
                        float q = pre[i];
#pragma unroll
                        for (int j = i + 1; j < d; ++j) q = q + rr[j];
                        qv[i] = q;
                    }
                    Q = pre[d];
                } else {
                    float sum = gamma_of(C);
#pragma unroll
                    for (int i = 0; i < d; ++i) sum += rr[i];
#pragma unroll
                    for (int i = 0; i < d; ++i) qv[i] = satf<FMT>(sum - rr[i]);
                    Q = sum;
                }
                if constexpr (POST) Qr[C] = Q;
                const bool e = Q < 0.0f;
                const uint32_t ew = e ? 1u : 0u;
                eb |= (uint64_t)e << C;
                static_for<0, d>([&](auto Ic) {
                    constexpr int i = decltype(Ic)::value;
                    constexpr int R = S::T.col_R[C][i];
                    wreg2::lds_u8 *row = (wreg2::lds_u8 *)&sh.xq[B::V.first[C] + i][0];
                    *(wreg2::lds_f32 *)(row + ad[i]) = qv[i];
                    wreg2::lds_u32 *ea = (wreg2::lds_u32 *)&sh.eacc[0] + (ad[i] >> 2);
                    __hip_atomic_fetch_xor(ea, ew << R, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                });
                // one column's values live at a time
                __builtin_amdgcn_sched_barrier(0);
            });
            __syncthreads();
            // 3. own rows back: new messages, and the decisions of the
            //    variables this lane's checks meet
            static_for<C0, C1>([&](auto Cc) {
                constexpr int C = decltype(Cc)::value;
                static_for<0, S::T.col_deg[C]>([&](auto Ic) {
                    constexpr int i = decltype(Ic)::value;
                    constexpr int R = S::T.col_R[C][i];
                    constexpr int slot = R * DC + S::T.col_j[C][i];
                    m[slot] = sh.xq[B::V.first[C] + i][r];
                });
                __builtin_amdgcn_sched_barrier(0);
            });
            __builtin_amdgcn_sched_barrier(0);
        });

        // ---------------- stopping rule, outputs ------------------------------
        // the last batch's second barrier has ordered every XOR into this row
        const bool bad = ((sh.eacc[r] ^ sb) & ((1u << MB) - 1u)) != 0;
        const uint64_t badmask = ballot(bad);
        if (t == 0) sh.unsat[k & 1][w] = badmask != 0 ? 1u : 0u;
        __syncthreads();
        uint32_t any = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) any |= __builtin_amdgcn_readfirstlane(sh.unsat[k & 1][i]);
        const bool conv = any == 0;
        if ((a.early_stop && conv) || k == a.max_iters) {
            // this wave's rows of every column: words (L / 32) C + 2 w and
            // (L / 32) C + 2 w + 1 (a rolled loop from an opaque base: unrolled,
            // the compiler would hoist 34 output addresses out of the iteration
            // loop)
            uint64_t eo = uniform64((uint64_t)(err_shot + 2 * w));
            asm volatile("" : "+s"(eo));
            uint32_t *err = (uint32_t *)eo;
#pragma unroll 1
            for (int C = 0; C < NB; ++C) {
                const uint64_t mc = ballot(((eb >> C) & 1ull) != 0);
                if (t < 2) err[(L / 32) * C + t] = (uint32_t)(mc >> (32 * t));
            }
            if (threadIdx.x == 0) {
                a.conv[shot] = conv ? 1 : 0;
                if (a.iters) a.iters[shot] = (uint8_t)k;
            }
            if constexpr (POST) {
#pragma unroll
                for (int C = 0; C < NB; ++C) {
                    const float q = FMT == 0 ? Qr[C] : Qr[C] * Fmt<FMT>::post_scale;
                    a.post[shot * N + C * L + r] = q;
                }
            }
            return;
        }
    }
}

// One workgroup of L / 64 waves per shot; grid = batch.  Per-bit priors and
// the a-posteriori output need more live registers than 168 (three waves per
// SIMD) leave without spilling, so those variants run two waves per SIMD.
template <class S, int FMT, bool PER_BIT, bool POST, int L>
__global__ __launch_bounds__(L) __attribute__((amdgpu_waves_per_eu((!PER_BIT && !POST) ? 3 : 2)))
void k_wreg2(const DecodeArgs a) {
    constexpr int SW = S::MB * L / 32, EW = S::NB * L / 32;
    __shared__ wreg2::Lds<S, FMT, L> sh;
    const long shot = xcd_wave_index(blockIdx.x, gridDim.x);
    if (shot >= a.batch) return;                                   // workgroup-uniform
    if (a.only && a.only[shot] == 0) return;                       // workgroup-uniform
    wreg2_decode<S, FMT, PER_BIT, POST, L>(a, a.code, shot, a.syn + shot * SW, a.err + shot * EW, sh);
}

template <class S, int FMT, int L>
hipError_t launch_wreg2(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    const dim3 g((unsigned)a.batch), blk(L);
    if (k.per_bit) {
        if (k.post) hipLaunchKernelGGL((k_wreg2<S, FMT, true, true, L>), g, blk, 0, st, a);
        else hipLaunchKernelGGL((k_wreg2<S, FMT, true, false, L>), g, blk, 0, st, a);
    } else {
        if (k.post) hipLaunchKernelGGL((k_wreg2<S, FMT, false, true, L>), g, blk, 0, st, a);
        else hipLaunchKernelGGL((k_wreg2<S, FMT, false, false, L>), g, blk, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace qldpc
