// Workgroup-per-shot min-sum decoder (latency layout) for gfx950, flooding
// schedule (Section 2, Algorithm 1).
//
// One workgroup of NW wavefronts decodes one shot of a lifted code with
// L = 64 or 128.  A work item is one 64-row slice of a block row (check
// pass) or of a block column (variable pass).  Every wave runs a copy of the
// iteration loop specialised at compile time for its own items (chosen once,
// by its wave index), so within an iteration a wave executes straight-line
// code with constant LDS offsets and no branches over other waves' items:
// an unrolled chain over every item, in which each wave branches past the
// items of the others, made an iteration at 16 waves about a third slower
// on MI355X.
//
// Per iteration k:
//   A: check pass of iteration k; each block row also tests the decisions of
//      iteration k-1 (its rows' parity words against the syndrome, see
//      kBlockParityWords) and raises a flag on a violated check;
//   barrier; every wave reads the flag: all checks satisfied -> emit the
//      outputs of iteration k-1 and stop (the check pass just run only
//      overwrote messages, not e or Q);
//   B: variable pass, a posteriori, decisions (ballots to LDS, changes XORed
//      into the parity words);
//   barrier.
// After the last iteration one more test pass decides the convergence flag.
// Two barriers per iteration; flags are double buffered by iteration parity.
#pragma once
#include "decode_wave.h"

namespace qldpc {

// Owner wave of every variable-pass item (a 64-row slice of a block column)
// and its slot among that wave's items.  Longest processing time first: the
// degree-5 columns are placed before the degree-3 ones, each on the wave with
// the least work so far, so that the slowest wave, which every iteration
// waits for at the barrier, carries as little as possible (9 edge slices per
// iteration at L = 64 with 16 waves, against 11 round robin).
template <class S, int L, int NW>
struct VnPlan {
    static constexpr int PPL = L / 64, ITEMS = S::NB * PPL;
    int owner[ITEMS];
    int slot[ITEMS];
    int per_wave;   // most items any wave holds
};

template <class S, int L, int NW>
constexpr VnPlan<S, L, NW> make_vn_plan() {
    using P = VnPlan<S, L, NW>;
    P p{};
    int load[NW] = {}, count[NW] = {};
    for (int deg = kMaxDv; deg >= 1; --deg)
        for (int it = 0; it < P::ITEMS; ++it) {
            if (S::T.col_deg[it / P::PPL] != deg) continue;
            int best = 0;
            for (int w = 1; w < NW; ++w)
                if (load[w] < load[best]) best = w;
            p.owner[it] = best;
            p.slot[it] = count[best]++;
            load[best] += deg;
        }
    p.per_wave = 0;
    for (int w = 0; w < NW; ++w) p.per_wave = count[w] > p.per_wave ? count[w] : p.per_wave;
    return p;
}

template <class S, int L, int NW>
struct VnPlanOf {
    static constexpr VnPlan<S, L, NW> P = make_vn_plan<S, L, NW>();
};

template <class S, int L, int FMT, int NW>
struct BlockLds {
    using msg_t = typename Fmt<FMT>::msg_t;
    static constexpr int PPL = L / 64;
    static constexpr size_t msg_bytes = (size_t)S::SLOTS * L * sizeof(msg_t);
    static constexpr size_t e_off = (msg_bytes + 15) & ~size_t(15);   // uint64 [NB][PPL]
    static constexpr size_t f_off = e_off + (size_t)S::NB * PPL * 8;  // uint32 flags[2]
    static constexpr size_t s_off = f_off + 16;                          // uint32 syndrome words
    static constexpr size_t a_off = (s_off + (((size_t)S::MB * L + 31) / 32) * 4 + 15) & ~size_t(15);
    static constexpr size_t bytes = a_off + (size_t)L * 4;               // uint32 check-row parity [L]
};

// Syndrome test by check-row parity words: the variable pass XORs every
// change of a decision into the word of each check row the variable meets
// (bit R for block row R, an LDS atomic per edge, skipped for an item where
// no decision of the wave changed), so after iteration k word row holds bit R
// = the parity of check (R, row) under the decisions of iteration k.  The
// check pass of iteration k + 1 compares its own rows' words with the
// syndrome: a read and three VALU per item instead of d rotated ballots.
constexpr bool kBlockParityWords = true;

// Decodes shot `shot` of the code whose shift table is `code_table` (its
// syndrome words at syn, error words to err; priors, flags and posteriors
// indexed by shot) with the whole workgroup.  a.code, a.syn and a.err are not
// used: the mixed-code path passes each shot's own table and ragged offsets.
// `lds` holds BlockLds<S, L, FMT, NW>::bytes.  Every thread of the workgroup
// must call it.
template <class S, int L, int FMT, int NW, bool PER_BIT, bool POST>
__device__ __forceinline__ void block_decode(const DecodeArgs &a, const DevCode *code_table, const long shot,
                                             const uint32_t *syn, uint32_t *err, unsigned char *lds) {
    using namespace wave;
    static_assert(L == 64 || L == 128, "block layout needs L >= 64");
    using Lay = BlockLds<S, L, FMT, NW>;
    using msg_t = typename Fmt<FMT>::msg_t;
    using prior_t = typename Fmt<FMT>::prior_t;
    using acc_t = typename std::conditional<FMT == 0, float, int>::type;
    constexpr int MB = S::MB, NB = S::NB, DC = S::DC, PPL = L / 64;
    constexpr int N = NB * L;
    constexpr int SW = (MB * L + 31) / 32, EW = (NB * L + 31) / 32;
    constexpr int CN_ITEMS = MB * PPL, VN_ITEMS = NB * PPL;
    using Plan = VnPlanOf<S, L, NW>;
    constexpr int VN_PER_WAVE = Plan::P.per_wave;
    static_assert(VN_PER_WAVE <= 32, "one bit per variable item of a wave");

    msg_t *msg = reinterpret_cast<msg_t *>(lds);
    uint64_t *emask = reinterpret_cast<uint64_t *>(lds + Lay::e_off);
    uint32_t *flag = reinterpret_cast<uint32_t *>(lds + Lay::f_off);
    uint32_t *rowpar = reinterpret_cast<uint32_t *>(lds + Lay::a_off);
    constexpr bool XT = kBlockParityWords;

    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const CodePtr code = const_code(code_table);
    uint32_t *synw = reinterpret_cast<uint32_t *>(lds + Lay::s_off);

    // the shot's syndrome words are read from memory once per workgroup (the
    // latency path reads them across the bus) and shared through LDS
    for (int w = threadIdx.x; w < SW; w += 64 * NW) synw[w] = syn[w];
    // priors of this wave's variable items (canonicalised: no message is -0.0)
    acc_t gam[PER_BIT ? VN_PER_WAVE : 1];
    if constexpr (!PER_BIT) {
        gam[0] = (acc_t) static_cast<const prior_t *>(a.prior)[shot];
        if constexpr (FMT == 0) gam[0] = gam[0] + 0.0f;
    } else {
        static_for<0, VN_ITEMS>([&](auto Ic) {
            constexpr int it = decltype(Ic)::value;
            if (Plan::P.owner[it] == wv) {
                constexpr int C = it / PPL, h = it % PPL;
                acc_t v = (acc_t) static_cast<const prior_t *>(a.prior)[shot * N + C * L + lane + 64 * h];
                if constexpr (FMT == 0) v = v + 0.0f;
                gam[Plan::P.slot[it]] = v;
            }
        });
    }
    auto gamma_of = [&](int it) -> acc_t { return PER_BIT ? gam[Plan::P.slot[it]] : gam[0]; };

    // q^(0) = gamma on every edge: each wave initialises its variable items
    static_for<0, VN_ITEMS>([&](auto Ic) {
        constexpr int it = decltype(Ic)::value;
        if (Plan::P.owner[it] == wv) {
            constexpr int C = it / PPL, h = it % PPL;
            const acc_t gm = gamma_of(it);
            static_for<0, S::T.col_deg[C]>([&](auto Jc) {
                constexpr int i = decltype(Jc)::value;
                constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                msg[slot * L + vn_index<L>(lane, h, (uint32_t)code->shift[slot])] = (msg_t)gm;
            });
        }
    });
    if (threadIdx.x == 0) {
        flag[0] = 0;
        flag[1] = 0;
    }
    if constexpr (XT) {
        for (int i = threadIdx.x; i < L; i += 64 * NW) rowpar[i] = 0;   // decisions of iteration 0: all 0
    }
    uint32_t eprev = 0;   // bit slot: this lane's decision of VN item slot in the last iteration
    acc_t Qr[POST ? VN_PER_WAVE : 1];
    __syncthreads();

    // syndrome bits of the checks this lane owns in each block row
    uint32_t sb[PPL];
#pragma unroll
    for (int h = 0; h < PPL; ++h) {
        sb[h] = 0;
#pragma unroll
        for (int R = 0; R < MB; ++R) {
            const int m = R * L + lane + 64 * h;
            sb[h] |= ((synw[m >> 5] >> (m & 31)) & 1u) << R;
        }
    }

    auto emit = [&](auto Wc, int k, bool conv) {
        constexpr int W = decltype(Wc)::value;
        // e words straight from the ballots; conv / iters by thread 0
        for (int w = threadIdx.x; w < EW; w += 64 * NW) {
            const uint64_t m = emask[(w * 32) / 64];
            err[w] = (uint32_t)(m >> ((w * 32) % 64));
        }
        if (threadIdx.x == 0) {
            a.conv[shot] = conv ? 1 : 0;
            if (a.iters) a.iters[shot] = (uint8_t)k;
        }
        if constexpr (POST) {
            static_for<0, VN_ITEMS>([&](auto Ic) {
                constexpr int it = decltype(Ic)::value;
                if constexpr (Plan::P.owner[it] == W) {
                    constexpr int C = it / PPL, h = it % PPL;
                    acc_t Q = Qr[Plan::P.slot[it]];
                    float qv;
                    if constexpr (FMT == 0) qv = Q;
                    else qv = (float)Q * Fmt<FMT>::post_scale;
                    a.post[shot * N + C * L + lane + 64 * h] = qv;
                }
            });
        }
    };

    // syndrome test of the last decisions; raises flag[par] on a violation
    auto test_rows = [&](auto Wc, int par) {
        constexpr int W = decltype(Wc)::value;
        if constexpr (XT) {
            bool bad = false;
            static_for<0, CN_ITEMS>([&](auto Ic) {
                constexpr int it = decltype(Ic)::value;
                if constexpr (it % NW == W) {
                    constexpr int R = it / PPL, h = it % PPL;
                    bad |= (((rowpar[lane + 64 * h] ^ sb[h]) >> R) & 1u) != 0;
                }
            });
            if (ballot(bad) != 0 && lane == 0) atomicOr(&flag[par], 1u);
            return;
        }
        static_for<0, CN_ITEMS>([&](auto Ic) {
            constexpr int it = decltype(Ic)::value;
            if constexpr (it % NW == W) {
                constexpr int R = it / PPL, h = it % PPL;
                uint64_t c = ballot(((sb[h] >> R) & 1u) != 0);
                static_for<0, DC>([&](auto Jc) {
                    constexpr int j = decltype(Jc)::value;
                    constexpr int C = S::T.slot_bc[R][j];
                    const uint32_t s = (uint32_t)code->shift[R * DC + j];
                    if constexpr (L == 64) {
                        const uint64_t e = emask[C];
                        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)e);
                        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(e >> 32));
                        c ^= seg_rotr<64>(((uint64_t)hi << 32) | lo, s, 0);
                    } else {
                        const uint64_t e0 = emask[C * PPL], e1 = emask[C * PPL + 1];
                        uint64_t lo, hi;
                        rotr128(e0, e1, s, lo, hi);
                        c ^= (h == 0) ? lo : hi;
                    }
                });
                if (c != 0 && lane == 0) atomicOr(&flag[par], 1u);
            }
        });
    };

    // the iteration loop, specialised for wave W's items
    auto run = [&](auto Wc) {
        constexpr int W = decltype(Wc)::value;
        int k = 1;
        for (; k <= a.max_iters; ++k) {
            // ---- A: check pass of iteration k, test of iteration k-1 ------------
            static_for<0, CN_ITEMS>([&](auto Ic) {
                constexpr int it = decltype(Ic)::value;
                if constexpr (it % NW == W) {
                    constexpr int R = it / PPL, h = it % PPL;
                    const uint32_t P = sb[h] << (31 - R);
                    if constexpr (FMT == 0) {
                        float v[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j) v[j] = msg[(R * DC + j) * L + lane + 64 * h];
                        cn_f32<DC>(v, P, a.alpha);
#pragma unroll
                        for (int j = 0; j < DC; ++j) msg[(R * DC + j) * L + lane + 64 * h] = v[j];
                    } else {
                        int v[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j) v[j] = msg[(R * DC + j) * L + lane + 64 * h];
                        cn_fx<DC>(v, P, a.alpha_num, a.alpha_shift);
#pragma unroll
                        for (int j = 0; j < DC; ++j) msg[(R * DC + j) * L + lane + 64 * h] = (msg_t)v[j];
                    }
                }
            });
            if (k > 1 && a.early_stop) test_rows(Wc, k & 1);
            __syncthreads();
            if (k > 1 && a.early_stop && __builtin_amdgcn_readfirstlane(flag[k & 1]) == 0) {   // uniform
                emit(Wc, k - 1, true);
                return;
            }
            // ---- B: variable pass, a posteriori, decisions ----------------------
            static_for<0, VN_ITEMS>([&](auto Ic) {
                constexpr int it = decltype(Ic)::value;
                if constexpr (Plan::P.owner[it] == W) {
                    constexpr int C = it / PPL, h = it % PPL;
                    constexpr int d = S::T.col_deg[C];
                    acc_t r[d];
                    int idx[d], row[d];
                    static_for<0, d>([&](auto Jc) {
                        constexpr int i = decltype(Jc)::value;
                        constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                        row[i] = vn_index<L>(lane, h, (uint32_t)code->shift[slot]);
                        idx[i] = slot * L + row[i];
                        r[i] = (acc_t)msg[idx[i]];
                    });
                    acc_t Q;
                    if constexpr (FMT == 0) {
                        float pre[d + 1];
                        pre[0] = gamma_of(it);
#pragma unroll
                        for (int i = 0; i < d; ++i) pre[i + 1] = pre[i] + r[i];
#pragma unroll
                        for (int i = 0; i < d; ++i) {
                            float q = pre[i];
#pragma unroll
                            for (int j = i + 1; j < d; ++j) q = q + r[j];
                            msg[idx[i]] = q;
                        }
                        Q = pre[d];
                    } else {
                        int sum = gamma_of(it);
#pragma unroll
                        for (int i = 0; i < d; ++i) sum += r[i];
#pragma unroll
                        for (int i = 0; i < d; ++i) msg[idx[i]] = (msg_t)sat<FMT>(sum - r[i]);
                        Q = sum;
                    }
                    if constexpr (POST) Qr[Plan::P.slot[it]] = Q;
                    const bool e = Q < (acc_t)0;
                    const uint64_t m = ballot(e);
                    if (lane == 0) emask[C * PPL + h] = m;
                    // without early stop only the last iteration's decisions are
                    // tested: eprev stays 0 until then, so that iteration XORs the
                    // whole decision vector into the (still zero) parity words
                    if constexpr (XT) {
                        constexpr int sl = Plan::P.slot[it];
                        const bool chg = e != (((eprev >> sl) & 1u) != 0);
                        if ((a.early_stop || k == a.max_iters) && ballot(chg) != 0) {   // wave-uniform
                            const uint32_t cw = chg ? 1u : 0u;
                            static_for<0, d>([&](auto Jc) {
                                constexpr int i = decltype(Jc)::value;
                                constexpr int R = S::T.col_R[C][i];
                                __hip_atomic_fetch_xor(&rowpar[row[i]], cw << R, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                            });
                            eprev ^= cw << sl;
                        }
                    }
                }
            });
            if (threadIdx.x == 0) flag[(k + 1) & 1] = 0;
            __syncthreads();
        }
        // after the last iteration: one more test decides the flag
        --k;
        test_rows(Wc, (k + 1) & 1);
        __syncthreads();
        emit(Wc, k, __builtin_amdgcn_readfirstlane(flag[(k + 1) & 1]) == 0);
    };
    static_for<0, NW>([&](auto Wc) {
        if (wv == decltype(Wc)::value) run(Wc);
    });
}

// Waves per SIMD the throughput kernel asks the register allocator for: an
// 8-wave workgroup with integer messages needs at most half of LDS per
// compute unit, so three workgroups fit if each wave stays within 80 VGPRs
// (the per-edge addresses the loop keeps otherwise take it to 133).
template <int L, int FMT, int NW>
constexpr int block_waves() { return (NW == 8 && FMT != 0) ? 4 : 1; }

template <class S, int L, int FMT, int NW, bool PER_BIT, bool POST>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(block_waves<L, FMT, NW>())))
void k_block(const DecodeArgs a) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[BlockLds<S, L, FMT, NW>::bytes];
    const long shot = blockIdx.x;
    if (a.only && a.only[shot] == 0) return;   // uniform over the workgroup
    constexpr int SW = (S::MB * L + 31) / 32, EW = (S::NB * L + 31) / 32;
    block_decode<S, L, FMT, NW, PER_BIT, POST>(a, a.code, shot, a.syn + shot * SW, a.err + shot * EW, lds);
}

template <class S, int L, int FMT, int NW, bool PB, bool PO>
hipError_t launch_block_one(const DecodeArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((k_block<S, L, FMT, NW, PB, PO>), dim3((unsigned)a.batch), dim3(64 * NW), 0, st, a);
    return hipGetLastError();
}

template <class S, int L, int FMT, int NW>
hipError_t launch_block(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.per_bit)
        return k.post ? launch_block_one<S, L, FMT, NW, true, true>(a, st)
                      : launch_block_one<S, L, FMT, NW, true, false>(a, st);
    return k.post ? launch_block_one<S, L, FMT, NW, false, true>(a, st)
                  : launch_block_one<S, L, FMT, NW, false, false>(a, st);
}

}  // namespace qldpc
