// Wavefront-per-shot min-sum decoder (throughput layout) for gfx950.
//
// Method: syndrome-based normalized min-sum, Section 2, Algorithm 1, in two
// schedules: flooding (all check nodes, then all variable nodes) and
// row-layered (block row by block row, a-posteriori values updated in place).
//
// Mapping.  The code is quasi-cyclic: a pattern of L x L circulants fixed at
// compile time, with run-time shifts.  One wavefront decodes 64 / L shots
// (L <= 64) or one shot (L = 128).  Lane t of a shot's segment owns row t of
// every circulant: check (R, t) of each block row R and variable (C, t) of
// each block column C.  Check (R, t) meets variable (C, (t + a) mod L)
// through block (R, C) = P^a, so a check-side access is lane-contiguous and
// a variable-side access is the same row rotated by a: both are free of LDS
// bank conflicts, and every address offset except the rotation is constant.
//
// LDS state per wave:
//   flooding: msg[(R * 8 + j) * ROW + lane], one entry per edge in CSR order,
//             holding q before a check pass and r after it (each entry is
//             read and written by exactly one lane per pass: in place);
//   layered:  r per edge (same layout) and the posterior Q[C * ROW + lane].
// ROW = 64 lanes (x2 circulant rows per lane at L = 128).
//
// Decisions and the syndrome test.  e_n = [Q_n < 0] of block column C is a
// 64-bit ballot.  Block row R accumulates s_R xor rot(e_C, a) over its 8
// blocks in scalar registers (a segment-wise rotation of the ballot by the
// circulant shift); the shot has converged when every accumulator is zero.
//
// Numerics.  FP32 follows a fixed order: excluded sums left to right from
// gamma_n in increasing check index, alpha * min rounded once, no
// contraction.  Priors are canonicalised with + 0.0f so no message is -0.0;
// the raw sign bit of q is then [q < 0] and the sign product is an XOR of
// sign bits.  Integer formats (int8 with Q4 priors, int16 with Q8 priors):
// |q| in [0, qmax], r = sign * ((num * min) >> sh), integer sums exact, q
// saturated to [-qmax, qmax] with qmax = 127 or 32767.
#pragma once
#include <stdint.h>

#include "kernels.h"
#include "shapes.h"

namespace qldpc {

// Scheduling knobs of the unrolled passes, per message format (measured on
// MI355X at L = 64, 65536 shots):
//  - sched group: a scheduling barrier after every G block rows (check pass)
//    and every G column batches (variable pass) bounds how far the compiler
//    hoists LDS loads, i.e. the registers a wave needs.  int8 kernels hold
//    little LDS and gain occupancy from it (11.9 -> 22 M syndromes/s); the
//    FP32 kernels are LDS-occupancy bound and lose ILP from it.  0 = none.
//  - variable-pass batch: block columns whose messages are all loaded
//    before any is overwritten (see the variable pass).
//  - wave cap: the most waves per SIMD the register allocation targets.
template <int FMT> struct Knobs;
template <> struct Knobs<0> { static constexpr int sched_group = 0, vn_batch = 4, wave_cap = 1; };
template <> struct Knobs<1> { static constexpr int sched_group = 1, vn_batch = 2, wave_cap = 4; };
template <> struct Knobs<2> { static constexpr int sched_group = 1, vn_batch = 2, wave_cap = 4; };
// Register-resident messages (see wave_decode): the variable pass loads the
// messages of 4 block columns before it writes any (their rotated reads then
// overlap), with a scheduling barrier after every batch, which keeps the
// compiler from interleaving batches and so bounds the scalar working set
// (shifts, rotated ballots).  Measured on MI355X at L = 64, 65536 shots, FP32
// flooding: 32.9 M syndromes/s with one column per batch and no barrier,
// 35.9 M with the barrier, 37.2 M with the barrier and 4 columns per batch.
struct RegKnobs { static constexpr int sched_group = 1, vn_batch = 4; };

template <int FMT>
__device__ __forceinline__ void sched_group_end(int idx) {
    constexpr int g = Knobs<FMT>::sched_group;
    if constexpr (g > 0) {
        if ((idx + 1) % g == 0) __builtin_amdgcn_sched_barrier(0);
    }
}

template <class S, int L>
struct Geo {
    static constexpr int SEG = L < 64 ? L : 64;      // lanes per shot
    static constexpr int SPW = 64 / SEG;             // shots per wave
    static constexpr int PPL = L > 64 ? L / 64 : 1;  // circulant rows per lane
    static constexpr int ROW = 64 * PPL;             // entries per slot row
    static constexpr int N = S::NB * L;
    static constexpr int SW = (S::MB * L + 31) / 32;  // syndrome words per shot
    static constexpr int EW = (S::NB * L + 31) / 32;  // error words per shot
    static constexpr uint64_t SEGMASK = L >= 64 ? ~0ull : ((1ull << L) - 1);
};

// Message formats: 0 = FP32; 1 = int8 messages, Q4 priors; 2 = int16
// messages, Q8 priors (the reduced-precision integer types of Section 3,
// Table 1).  q_t holds a layered a-posteriori value: |Q| <= qmax + d_v
// (3 qmax >> 2), which needs 16 bits for int8 and 32 for int16.  The reported
// posterior is Q * post_scale.
template <int FMT> struct Fmt;
template <> struct Fmt<0> {
    using msg_t = float; using q_t = float; using prior_t = float;
    static constexpr int qmax = 0;
    static constexpr float post_scale = 1.0f;
};
template <> struct Fmt<1> {
    using msg_t = int8_t; using q_t = int16_t; using prior_t = int8_t;
    static constexpr int qmax = 127;
    static constexpr float post_scale = 0.0625f;
};
template <> struct Fmt<2> {
    using msg_t = int16_t; using q_t = int32_t; using prior_t = int16_t;
    static constexpr int qmax = 32767;
    static constexpr float post_scale = 0.00390625f;
};

// LDS of one wave.  REG: messages live in registers; only the staging of
// the packed decisions remains.
template <class S, int L, int FMT, int SCHED, int NG = 1, bool REG = false>
struct WaveLds {
    using G = Geo<S, L>;
    using msg_t = typename Fmt<FMT>::msg_t;
    using q_t = typename Fmt<FMT>::q_t;
    static constexpr int H = L <= 64 ? NG : L / 64;
    static constexpr int ROW = 64 * H;
    static constexpr int MSG = REG ? 0 : S::SLOTS * ROW;
    static constexpr int QN = (SCHED == 1 && !REG) ? S::NB * ROW : 0;
    static constexpr size_t msg_bytes = MSG * sizeof(msg_t);
    static constexpr size_t q_off = (msg_bytes + 15) & ~size_t(15);
    static constexpr size_t e_off = (q_off + QN * sizeof(q_t) + 15) & ~size_t(15);
    static constexpr size_t bytes = e_off + (L <= 64 ? NG : 1) * G::SPW * G::EW * 4;
};

namespace wave {

// Rotate every L-bit segment of a ballot right by s: bit t of a segment
// becomes bit (t + s) mod L of the same segment.  `low` has the low L - s
// bits of every segment set.
template <int L>
__device__ __forceinline__ uint64_t seg_rotr(uint64_t m, uint32_t s, uint64_t low) {
    if constexpr (L == 64) {
        return (m >> s) | (m << ((64u - s) & 63u));
    } else {
        return ((m >> s) & low) | ((m << (L - s)) & ~low);
    }
}

// 128-bit rotate right (L = 128: positions 0..63 in lo, 64..127 in hi).
__device__ __forceinline__ void rotr128(uint64_t lo, uint64_t hi, uint32_t s, uint64_t &olo,
                                        uint64_t &ohi) {
    if (s >= 64u) {
        const uint64_t t = lo;
        lo = hi;
        hi = t;
        s -= 64u;
    }
    olo = (lo >> s) | ((hi << 1) << (63u - s));
    ohi = (hi >> s) | ((lo << 1) << (63u - s));
}

// gfx950's three-input bitwise operation: bit i of the result is f(bit i of
// a, bit i of b, bit i of c), f given by its truth table TT (the table of a
// function is that function applied to 0xF0, 0xCC and 0xAA).
template <uint32_t TT>
__device__ __forceinline__ uint32_t bitop3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}
constexpr uint32_t kXor3 = (0xF0u ^ 0xCCu ^ 0xAAu) & 0xFFu;       // a ^ b ^ c
constexpr uint32_t kXorAnd = (0xF0u ^ (0xCCu & 0xAAu)) & 0xFFu;   // a ^ (b & c)
constexpr uint32_t kOrAnd = (0xF0u | (0xCCu & 0xAAu)) & 0xFFu;    // a | (b & c)
constexpr uint32_t kSign = 0x80000000u;

__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float ubits(uint32_t x) { return __uint_as_float(x); }
__device__ __forceinline__ uint64_t ballot(bool b) { return __ballot(b); }

// Position inside a slot row of the entry that variable position
// (lane + 64 h) reaches through a block of shift s (check = var - s).
template <int L>
__device__ __forceinline__ int vn_index(int lane, int h, uint32_t s) {
    if constexpr (L <= 64) {
        return (int)(((uint32_t)lane - s) & (uint32_t)(L - 1)) | (lane & ~(L - 1));
    } else {
        return (int)(((uint32_t)(lane + 64 * h) - s) & (uint32_t)(L - 1));
    }
}

// Position inside a block-column row of the variable that check position
// (lane + 64 h) reaches through a block of shift s (var = check + s).
template <int L>
__device__ __forceinline__ int cn_index(int lane, int h, uint32_t s) {
    if constexpr (L <= 64) {
        return (int)(((uint32_t)lane + s) & (uint32_t)(L - 1)) | (lane & ~(L - 1));
    } else {
        return (int)(((uint32_t)(lane + 64 * h) + s) & (uint32_t)(L - 1));
    }
}

// ---- check-node rule, FP32 (Algorithm 1): r_j = (-1)^{s + sum_{i != j} neg_i}
//      * fl(alpha * min_{i != j} |q_i|).  P carries s in bit 31 on entry.
// Sign parity of a check: bit 31 of P ^ v_0 ^ ... ^ v_{DC-1} (three-input
// XORs; the lower bits are don't-cares).
template <int DC>
__device__ __forceinline__ uint32_t sign_parity(const float (&v)[DC], uint32_t P) {
    int j = 0;
#pragma unroll
    for (; j + 1 < DC; j += 2) P = bitop3<kXor3>(P, fbits(v[j]), fbits(v[j + 1]));
    if (j < DC) P ^= fbits(v[j]);
    return P;
}

// The outgoing messages of a check from its two candidate magnitudes A1
// (not the minimum edge) and A2 (the minimum edge): the check sign P is put
// on both once, then each edge flips it by its own sign bit, so an edge costs
// a compare, a select and one three-input operation.
template <int DC>
__device__ __forceinline__ void cn_emit(float (&v)[DC], uint32_t P, float m1, float A1, float A2) {
    const uint32_t B1 = bitop3<kOrAnd>(fbits(A1), P, kSign);
    const uint32_t B2 = bitop3<kOrAnd>(fbits(A2), P, kSign);
    // |q_j| == min1: j is the (or a tied) minimum; the excluded minimum is
    // min2 (equal to min1 on a tie).  All compares first, so that no select
    // waits on the compare just before it.
    bool isMin[DC];
#pragma unroll
    for (int j = 0; j < DC; ++j) isMin[j] = fabsf(v[j]) == m1;
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        const uint32_t b = isMin[j] ? B2 : B1;
        v[j] = ubits(bitop3<kXorAnd>(b, fbits(v[j]), kSign));
    }
}

template <int DC>
__device__ __forceinline__ void cn_f32(float (&v)[DC], uint32_t P, float alpha) {
    float m1 = fminf(fabsf(v[0]), fabsf(v[1]));
    float m2 = fmaxf(fabsf(v[0]), fabsf(v[1]));
#pragma unroll
    for (int j = 2; j < DC; ++j) {
        m2 = __builtin_amdgcn_fmed3f(m1, m2, fabsf(v[j]));
        m1 = fminf(m1, fabsf(v[j]));
    }
    P = sign_parity<DC>(v, P);
    float A1 = alpha * m1;
    float A2 = alpha * m2;
    // two products per check: keep the compiler from moving the multiply
    // behind the per-edge select below (one product per edge)
    asm volatile("" : "+v"(A1), "+v"(A2));
    cn_emit<DC>(v, P, m1, A1, A2);
}

// ---- check-node rule, integer formats: magnitudes in [0, qmax], alpha =
//      num / 2^sh applied to the magnitude and rounded down, before the sign.
template <int DC>
__device__ __forceinline__ void cn_fx(int (&v)[DC], uint32_t P, int num, int sh) {
    int a[DC];
#pragma unroll
    for (int j = 0; j < DC; ++j) a[j] = v[j] < 0 ? -v[j] : v[j];
    int m1 = min(a[0], a[1]);
    int m2 = max(a[0], a[1]);
#pragma unroll
    for (int j = 2; j < DC; ++j) {
        m2 = max(m1, min(m2, a[j]));   // med3(m1, m2, a_j) for m1 <= m2
        m1 = min(m1, a[j]);
    }
#pragma unroll
    for (int j = 0; j < DC; ++j) P ^= (uint32_t)v[j];
    const int A1 = (num * m1) >> sh;
    const int A2 = (num * m2) >> sh;
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        const int mag = (a[j] == m1) ? A2 : A1;
        v[j] = ((int)(P ^ (uint32_t)v[j]) < 0) ? -mag : mag;
    }
}

// Saturation of a message of an integer format to [-qmax, qmax].
template <int FMT>
__device__ __forceinline__ int sat(int x) {
    constexpr int Q = Fmt<FMT>::qmax;
    return min(Q, max(-Q, x));
}

// ---- integer formats on integer-valued FP32 lanes (register layout) -------
// Every value of the integer formats is an integer of magnitude below 2^24
// (|Q| <= qmax + 5 (3 qmax >> 2) < 2^18), so FP32 holds it, and sums and
// differences of such values, exactly.  alpha = num / 2^sh with num * |q| <
// 2^24, so fl(alpha * min) is exact and its floor is (num * min) >> sh.  The
// same values as cn_fx and sat, bit for bit, on the FP32 instructions, whose
// abs and negate operand modifiers the integer instructions lack.  No value
// is ever -0.0 (sums start from a converted integer prior), so the sign bit of
// q is [q < 0].
template <int DC>
__device__ __forceinline__ void cn_fxf(float (&v)[DC], uint32_t P, float alpha) {
    float m1 = fminf(fabsf(v[0]), fabsf(v[1]));
    float m2 = fmaxf(fabsf(v[0]), fabsf(v[1]));
#pragma unroll
    for (int j = 2; j < DC; ++j) {
        m2 = __builtin_amdgcn_fmed3f(m1, m2, fabsf(v[j]));
        m1 = fminf(m1, fabsf(v[j]));
    }
    P = sign_parity<DC>(v, P);
    float A1 = floorf(alpha * m1);
    float A2 = floorf(alpha * m2);
    asm volatile("" : "+v"(A1), "+v"(A2));
    cn_emit<DC>(v, P, m1, A1, A2);
}

template <int FMT>
__device__ __forceinline__ float satf(float x) {
    constexpr float Q = (float)Fmt<FMT>::qmax;
    return __builtin_amdgcn_fmed3f(-Q, x, Q);
}

// The value of lane 0, as a wave-uniform (scalar) value.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// The value `v` held by the lane whose byte address (4 * lane) is `addr`.
__device__ __forceinline__ float bperm(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ int bperm(int addr, int v) { return __builtin_amdgcn_ds_bpermute(addr, v); }
// Forward permute: the lane whose byte address (4 * lane) is `addr` receives
// `v` (addresses must form a permutation of the lanes).
__device__ __forceinline__ float fperm(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_permute(addr, __float_as_int(v)));
}

}  // namespace wave

// ---------------------------------------------------------------------------
// The decoder body: decodes the 64 / L (or 1) shots starting at shot_base.
// `lds` points to WaveLds<...>::bytes of this wave's LDS.
// ---------------------------------------------------------------------------
// Check rule with per-edge scales (neural min-sum): r_j = sgn_j * fl(w_j *
// excluded_min_j).  A weight may be negative: the product then carries its
// own sign bit, and the check sign flips it (XOR), as multiplying by sgn_j
// would.
namespace wave {
template <int DC>
__device__ __forceinline__ void cn_f32_weighted(float (&v)[DC], uint32_t P, const float (&wj)[DC]) {
    float m1 = fminf(fabsf(v[0]), fabsf(v[1]));
    float m2 = fmaxf(fabsf(v[0]), fabsf(v[1]));
#pragma unroll
    for (int j = 2; j < DC; ++j) {
        m2 = __builtin_amdgcn_fmed3f(m1, m2, fabsf(v[j]));
        m1 = fminf(m1, fabsf(v[j]));
    }
    P = sign_parity<DC>(v, P);
    // the check sign on both candidate minima: fl(w * (+-m)) = +-fl(w * m)
    const float M1 = ubits(bitop3<kOrAnd>(fbits(m1), P, kSign));
    const float M2 = ubits(bitop3<kOrAnd>(fbits(m2), P, kSign));
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        const float wm = wj[j] * ((fabsf(v[j]) == m1) ? M2 : M1);
        v[j] = ubits(bitop3<kXorAnd>(fbits(wm), fbits(v[j]), kSign));
    }
}

// The DC weights of check (R, pos) at iteration k: w[k][(R*L + pos)*DC + j].
template <int L, int DC>
__device__ __forceinline__ void load_weights(const float *__restrict__ w, int k, int nnz, int R, int pos,
                                             float (&wj)[DC]) {
    const float4 *p = reinterpret_cast<const float4 *>(w + (size_t)k * nnz + (size_t)(R * L + pos) * DC);
#pragma unroll
    for (int q = 0; q < DC / 4; ++q) {
        const float4 x = p[q];
        wj[4 * q] = x.x;
        wj[4 * q + 1] = x.y;
        wj[4 * q + 2] = x.z;
        wj[4 * q + 3] = x.w;
    }
}
}  // namespace wave

// One 64-lane group of a wavefront: the shot it decodes (-1 = none) and
// where that shot's packed syndrome and error words live.
struct ShotRef {
    long shot;
    const uint32_t *syn;
    uint32_t *err;
};

// ---------------------------------------------------------------------------
// The decoder body.  A lane owns H "halves": for L = 128 the two circulant
// rows t and t + 64 of one shot; for L <= 64, NG independent 64-lane groups,
// each decoding its own 64 / L shots (ref[h] describes group h's segment of
// this lane).  `lds` points to WaveLds<S, L, FMT, SCHED, NG, REG>::bytes.
//
// REG (L <= 64, one group): the lane's entry of every slot row is kept in a
// register array m[slot] instead of LDS (integer messages as 32-bit integers).  Flooding: the check pass
// works on registers only; the variable pass fetches the entry a variable
// reaches through a block of shift s from lane (t - s) mod L with a
// cross-lane permute (ds_bpermute) and returns its new message to lane
// (t + s) mod L the same way.  Layered: the check messages r never move;
// the lane's a-posteriori values Q of all 34 block columns are registers
// too, and each layer fetches the Q its check sees through shift s from lane
// (t + s) mod L and returns the updated Q to lane (t - s) mod L.  Values and
// the order of every operation are those of the LDS form; only where the
// messages are kept differs.
// ---------------------------------------------------------------------------
// WEIGHTED: 0 = alpha; 1 = per-edge weights in every iteration (neural
// min-sum); 2 = weights in iterations 1..a.weight_iters, alpha after (plain
// min-sum continuing from the neural messages).
template <class S, int L, int FMT, int SCHED, bool PER_BIT, bool POST, int WEIGHTED, int NG, bool REG = false>
__device__ __forceinline__ void wave_decode(const DecodeArgs &a, const DevCode *__restrict__ code,
                                            const ShotRef (&ref)[NG], unsigned char *lds) {
    using namespace wave;
    using G = Geo<S, L>;
    using Lay = WaveLds<S, L, FMT, SCHED, NG, REG>;
    using msg_t = typename Fmt<FMT>::msg_t;
    using q_t = typename Fmt<FMT>::q_t;
    using prior_t = typename Fmt<FMT>::prior_t;
    // REG: integer formats run on integer-valued FP32 lanes (cn_fxf, satf)
    constexpr bool FXF = REG && FMT != 0;
    using acc_t = typename std::conditional<FMT == 0 || FXF, float, int>::type;
    static_assert(L <= 64 || NG == 1, "L = 128 uses both halves for one shot");
    static_assert(!REG || (L <= 64 && NG == 1 && !(WEIGHTED && (SCHED == 1 || FMT != 0))),
                  "register-resident messages: L <= 64, one group");
    constexpr bool GRP = L <= 64;                 // halves are independent groups
    constexpr int H = GRP ? NG : L / 64;          // halves per lane
    constexpr int MB = S::MB, NB = S::NB, DC = S::DC, ROW = 64 * H;

    msg_t *msg = reinterpret_cast<msg_t *>(lds);
    q_t *Qs = reinterpret_cast<q_t *>(lds + Lay::q_off);
    uint32_t *ebuf = reinterpret_cast<uint32_t *>(lds + Lay::e_off);

    const int lane = threadIdx.x & 63;
    const int g = lane / G::SEG;
    const int p = lane % G::SEG;
    auto grp = [](int h) { return GRP ? h : 0; };
    auto posoff = [](int h) { return GRP ? 0 : 64 * h; };   // circulant row offset of half h
    // LDS row index of the entry that variable position (lane, half h)
    // reaches through a block of shift s (check = var - s), and back.
    auto vn_at = [&](int h, uint32_t s) -> int {
        if constexpr (GRP) return 64 * h + ((int)(((uint32_t)lane - s) & (uint32_t)(L - 1)) | (lane & ~(L - 1)));
        else return (int)(((uint32_t)(lane + 64 * h) - s) & (uint32_t)(L - 1));
    };
    auto cn_at = [&](int h, uint32_t s) -> int {
        if constexpr (GRP) return 64 * h + ((int)(((uint32_t)lane + s) & (uint32_t)(L - 1)) | (lane & ~(L - 1)));
        else return (int)(((uint32_t)(lane + 64 * h) + s) & (uint32_t)(L - 1));
    };
    // REG: messages in registers, shifts read as scalars, and the byte
    // addresses of the lanes (t - s) and (t + s) mod L within the segment.
    // The table pointer is re-derived opaquely for every batch of block
    // columns, so the compiler reloads each batch's shifts (scalar-cache
    // hits) instead of hoisting all 120 out of the loop into scalar registers
    // it does not have.
    acc_t m[REG ? S::SLOTS : 1];
    acc_t Qv[(REG && SCHED == 1) ? S::NB : 1];   // layered: this lane's Q of every block column
    const uint32_t lane4 = (uint32_t)lane << 2;
    CodePtr cpb = const_code(code);
    auto reload_table = [&]() {
        uint64_t v = (uint64_t)code;
        asm volatile("" : "+s"(v));
        cpb = (CodePtr)v;
    };
    auto shift_of = [&](int slot) -> uint32_t {
        if constexpr (REG) return (uint32_t)cpb->shift[slot];
        else return (uint32_t)code->shift[slot];
    };
    // (ds_bpermute selects lane (address / 4) mod 64 and ignores the higher
    // address bits, so for L = 64 the wrap needs no mask.)
    auto vn_src = [&](uint32_t s) -> int {
        if constexpr (L == 64) return (int)(lane4 - (s << 2));
        else return (int)(((lane4 - (s << 2)) & (uint32_t)(4 * L - 4)) | (lane4 & ~(uint32_t)(4 * L - 1)));
    };
    auto cn_src = [&](uint32_t s) -> int {
        if constexpr (L == 64) return (int)(lane4 + (s << 2));
        else return (int)(((lane4 + (s << 2)) & (uint32_t)(4 * L - 4)) | (lane4 & ~(uint32_t)(4 * L - 1)));
    };
    // REG flooding, edge i of block column C: the byte address of lane
    // (t + c) mod L = (t - s) mod L, whose check meets this lane's variable.
    // The variable pass reads the message there (ds_bpermute) and sends the
    // new one back to the same lane (ds_permute), one address for both.
    auto vn_lane = [&](int C, int i) -> int {
        // lane4 + 4c in one vector instruction from the scalar c
        const uint32_t c = (uint32_t)cpb->colrot[C][i].c;
        uint32_t d;
        asm("v_mad_u32_u24 %0, %1, 4, %2" : "=v"(d) : "s"(c), "v"(lane4));
        if constexpr (L == 64) return (int)d;
        else return (int)((d & (uint32_t)(4 * L - 4)) | (lane4 & ~(uint32_t)(4 * L - 1)));
    };

    bool valid[NG];
    bool any_valid = false;
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        valid[q] = ref[q].shot >= 0 && !(a.only && a.only[ref[q].shot] == 0);
        any_valid = any_valid || valid[q];
    }
    if (ballot(any_valid) == 0) return;   // nothing to decode in this wave (masked or past the batch)

    // Syndrome bits of this lane's checks: bit R of sb[h] = s of check R*L + p + posoff(h).
    uint32_t sb[H];
#pragma unroll
    for (int h = 0; h < H; ++h) {
        sb[h] = 0;
        if (valid[grp(h)]) {
#pragma unroll
            for (int R = 0; R < MB; ++R) {
                const int m = R * L + p + posoff(h);
                const uint32_t w = ref[grp(h)].syn[m >> 5];
                sb[h] |= ((w >> (m & 31)) & 1u) << R;
            }
        }
    }
    // Priors (FP32 canonicalised so that no message is -0.0).
    acc_t gam[PER_BIT ? NB * H : NG];
    {
        const prior_t *pr = static_cast<const prior_t *>(a.prior);
        if constexpr (PER_BIT) {
#pragma unroll
            for (int C = 0; C < NB; ++C)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    acc_t v = valid[grp(h)] ? (acc_t)pr[ref[grp(h)].shot * G::N + C * L + p + posoff(h)] : (acc_t)1;
                    if constexpr (FMT == 0) v = v + 0.0f;
                    gam[C * H + h] = v;
                }
        } else {
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                acc_t v = valid[q] ? (acc_t)pr[ref[q].shot] : (acc_t)1;
                if constexpr (FMT == 0) v = v + 0.0f;
                gam[q] = v;
            }
        }
    }
    auto gamma_of = [&](int C, int h) -> acc_t { return PER_BIT ? gam[C * H + h] : gam[grp(h)]; };

    // Initial state.  Flooding: q^(0) = gamma on every edge.  Layered: r = 0,
    // Q = gamma.
    if constexpr (SCHED == 0) {
        static_for<0, NB>([&](auto Cc) {
            constexpr int C = decltype(Cc)::value;
            static_for<0, S::T.col_deg[C]>([&](auto Ii) {
                constexpr int i = decltype(Ii)::value;
                constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                const uint32_t s = shift_of(slot);
                if constexpr (REG) {
                    // the check at position t of this slot sees variable t + s
                    m[slot] = PER_BIT ? bperm(cn_src(s), gamma_of(C, 0)) : gamma_of(C, 0);
                } else {
#pragma unroll
                    for (int h = 0; h < H; ++h) msg[slot * ROW + vn_at(h, s)] = (msg_t)gamma_of(C, h);
                }
            });
        });
    } else if constexpr (REG) {
        static_for<0, S::SLOTS>([&](auto Sc) { m[decltype(Sc)::value] = (acc_t)0; });
        static_for<0, NB>([&](auto Cc) { Qv[decltype(Cc)::value] = gamma_of(decltype(Cc)::value, 0); });
    } else {
#pragma unroll
        for (int sl = 0; sl < S::SLOTS; ++sl)
#pragma unroll
            for (int h = 0; h < H; ++h) msg[sl * ROW + lane + 64 * h] = (msg_t)0;
#pragma unroll
        for (int C = 0; C < NB; ++C)
#pragma unroll
            for (int h = 0; h < H; ++h) Qs[C * ROW + lane + 64 * h] = (q_t)gamma_of(C, h);
    }

    acc_t Qr[POST ? NB * H : 1];
    uint64_t eb[H];
    bool done[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) done[q] = !valid[q];

    for (int k = 1; k <= a.max_iters; ++k) {
        __builtin_amdgcn_wave_barrier();
        // Syndrome accumulators of the block rows, seeded with the rows'
        // syndrome ballots.  REG: seeded after the check pass from an opaque
        // copy of sb, so the ballots are re-derived every iteration instead
        // of being hoisted out of the loop, where they would pin 2 * MB scalar
        // registers for its whole length.
        uint64_t acc[MB][H];
        auto seed_acc = [&]() {
            uint32_t sbo[H];
#pragma unroll
            for (int h = 0; h < H; ++h) {
                sbo[h] = sb[h];
                if constexpr (REG) asm volatile("" : "+v"(sbo[h]));
            }
#pragma unroll
            for (int R = 0; R < MB; ++R)
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    acc[R][h] = ballot(((sbo[h] >> R) & 1u) != 0);
                }
        };
        if constexpr (!REG) seed_acc();
#pragma unroll
        for (int h = 0; h < H; ++h) eb[h] = 0;

        // REG: the wave's priority is raised for the variable pass (cross-lane
        // permutes and their dependent sums) and lowered for the check pass
        // (registers only), so a wave's permutes issue ahead of the other
        // waves' register work, which then fills the wait (37.1 -> 38.2-38.7 M
        // syndromes/s at L = 64; 23.0 -> 24.1 M with 16 fixed iterations).
        if constexpr (REG) __builtin_amdgcn_s_setprio(0);
        if constexpr (SCHED == 0) {
            // ---------------- check-node pass --------------------------------
#pragma unroll
            for (int R = 0; R < MB; ++R) {
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const uint32_t P = sb[h] << (31 - R);
                    if constexpr (FMT == 0) {
                        float v[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j)
                            v[j] = REG ? m[R * DC + j] : msg[(R * DC + j) * ROW + lane + 64 * h];
                        if constexpr (WEIGHTED == 2) {
                            if (k <= a.weight_iters) {   // uniform: neural iterations, then plain
                                float wj[DC];
                                load_weights<L, DC>(a.weights, k - 1, MB * L * DC, R, p + posoff(h), wj);
                                cn_f32_weighted<DC>(v, P, wj);
                            } else {
                                cn_f32<DC>(v, P, a.alpha);
                            }
                        } else if constexpr (WEIGHTED == 1) {
                            float wj[DC];
                            load_weights<L, DC>(a.weights, k - 1, MB * L * DC, R, p + posoff(h), wj);
                            cn_f32_weighted<DC>(v, P, wj);
                        } else {
                            cn_f32<DC>(v, P, a.alpha);
                        }
#pragma unroll
                        for (int j = 0; j < DC; ++j) {
                            if constexpr (REG) m[R * DC + j] = v[j];
                            else msg[(R * DC + j) * ROW + lane + 64 * h] = v[j];
                        }
                    } else if constexpr (FXF) {
                        float v[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j) v[j] = m[R * DC + j];
                        cn_fxf<DC>(v, P, a.alpha);
#pragma unroll
                        for (int j = 0; j < DC; ++j) m[R * DC + j] = v[j];
                    } else {
                        int v[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j)
                            v[j] = REG ? (int)m[R * DC + j] : (int)msg[(R * DC + j) * ROW + lane + 64 * h];
                        cn_fx<DC>(v, P, a.alpha_num, a.alpha_shift);
#pragma unroll
                        for (int j = 0; j < DC; ++j) {
                            if constexpr (REG) m[R * DC + j] = (acc_t)v[j];
                            else msg[(R * DC + j) * ROW + lane + 64 * h] = (msg_t)v[j];
                        }
                    }
                }
                sched_group_end<FMT>(R);
            }
            __builtin_amdgcn_wave_barrier();
        } else {
            // ---------------- layers: one block row at a time ----------------
            static_for<0, MB>([&](auto Rc) {
                constexpr int R = decltype(Rc)::value;
                if constexpr (REG) {
                    reload_table();
                    const uint32_t P = sb[0] << (31 - R);
                    acc_t v[DC], c[DC];
                    static_for<0, DC>([&](auto Jc) {
                        constexpr int j = decltype(Jc)::value;
                        constexpr int C = S::T.slot_bc[R][j];
                        // Q of the variable (C, t + s) this lane's check sees, minus the old r
                        v[j] = bperm(cn_src(shift_of(R * DC + j)), Qv[C]) - m[R * DC + j];
                        if constexpr (FMT == 0) c[j] = v[j];
                        else c[j] = satf<FMT>(v[j]);     // check-node input
                    });
                    if constexpr (FMT == 0) cn_f32<DC>(c, P, a.alpha);
                    else cn_fxf<DC>(c, P, a.alpha);
                    static_for<0, DC>([&](auto Jc) {
                        constexpr int j = decltype(Jc)::value;
                        constexpr int C = S::T.slot_bc[R][j];
                        m[R * DC + j] = c[j];
                        // the variable at position t + s receives the value of check t
                        Qv[C] = fperm(cn_src(shift_of(R * DC + j)), v[j] + c[j]);
                    });
                    return;
                }
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const uint32_t P = sb[h] << (31 - R);
                    int qi[DC];
                    acc_t v[DC], rold[DC];
                    static_for<0, DC>([&](auto Jc) {
                        constexpr int j = decltype(Jc)::value;
                        constexpr int C = S::T.slot_bc[R][j];
                        const uint32_t s = (uint32_t)code->shift[R * DC + j];
                        qi[j] = C * ROW + cn_at(h, s);
                        rold[j] = (acc_t)msg[(R * DC + j) * ROW + lane + 64 * h];
                    });
                    if constexpr (FMT == 0) {
#pragma unroll
                        for (int j = 0; j < DC; ++j) v[j] = Qs[qi[j]] - rold[j];
                        float c[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j) c[j] = v[j];
                        cn_f32<DC>(c, P, a.alpha);
#pragma unroll
                        for (int j = 0; j < DC; ++j) {
                            Qs[qi[j]] = v[j] + c[j];
                            msg[(R * DC + j) * ROW + lane + 64 * h] = c[j];
                        }
                    } else {
                        int c[DC];
#pragma unroll
                        for (int j = 0; j < DC; ++j) {
                            v[j] = (int)Qs[qi[j]] - rold[j];     // exact
                            c[j] = sat<FMT>(v[j]);                 // check-node input
                        }
                        cn_fx<DC>(c, P, a.alpha_num, a.alpha_shift);
#pragma unroll
                        for (int j = 0; j < DC; ++j) {
                            Qs[qi[j]] = (q_t)(v[j] + c[j]);
                            msg[(R * DC + j) * ROW + lane + 64 * h] = (msg_t)c[j];
                        }
                    }
                }
            });
            __builtin_amdgcn_wave_barrier();
        }

        if constexpr (REG) seed_acc();
        if constexpr (REG) __builtin_amdgcn_s_setprio(2);
        // ---------------- variable nodes, a posteriori, decision -------------
        // Block columns are processed Knobs::vn_batch at a time: every message
        // of the batch is loaded before any is overwritten, so the rotated
        // loads of a batch overlap instead of each column waiting for the
        // previous column's stores (the compiler cannot prove that rotated
        // addresses of different columns never alias).
        constexpr int VB = REG ? RegKnobs::vn_batch : Knobs<FMT>::vn_batch;
        static_for<0, (NB + VB - 1) / VB>([&](auto Bc) {
            constexpr int C0 = decltype(Bc)::value * VB;
            constexpr int NC = (C0 + VB <= NB) ? VB : NB - C0;
            if constexpr (REG) reload_table();
            acc_t rr[NC][H][kMaxDv];
            int ii[NC][H][kMaxDv];
            if constexpr (SCHED == 0) {
                static_for<0, NC>([&](auto Kc) {
                    constexpr int kc = decltype(Kc)::value;
                    constexpr int C = C0 + kc;
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        static_for<0, S::T.col_deg[C]>([&](auto Ii) {
                            constexpr int i = decltype(Ii)::value;
                            constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                            if constexpr (REG) {
                                rr[kc][h][i] = bperm(vn_lane(C, i), m[slot]);
                            } else {
                                ii[kc][h][i] = slot * ROW + vn_at(h, (uint32_t)code->shift[slot]);
                                rr[kc][h][i] = (acc_t)msg[ii[kc][h][i]];
                            }
                        });
                    }
                });
            }
            static_for<0, NC>([&](auto Kc) {
                constexpr int kc = decltype(Kc)::value;
                constexpr int C = C0 + kc;
                constexpr int d = S::T.col_deg[C];
                uint64_t mask[H];
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    acc_t Q;
                    if constexpr (SCHED == 0) {
                        const acc_t *r = rr[kc][h];
                        const int *idx = ii[kc][h];
                        if constexpr (FMT == 0) {
                            // prefix sums from gamma in increasing check order; the
                            // excluded sum of edge i continues the prefix before i
                            float pre[d + 1], qv[d];
                            pre[0] = gamma_of(C, h);
#pragma unroll
                            for (int i = 0; i < d; ++i) pre[i + 1] = pre[i] + r[i];
#pragma unroll
                            for (int i = 0; i < d; ++i) {
                                float q = pre[i];
#pragma unroll
                                for (int j = i + 1; j < d; ++j) q = q + r[j];
                                qv[i] = q;
                            }
                            if constexpr (REG) {
                                static_for<0, d>([&](auto Ii) {
                                    constexpr int i = decltype(Ii)::value;
                                    constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                                    m[slot] = fperm(vn_lane(C, i), qv[i]);
                                });
                            } else {
#pragma unroll
                                for (int i = 0; i < d; ++i) msg[idx[i]] = qv[i];
                            }
                            Q = pre[d];
                        } else if constexpr (FXF) {
                            // exact integer values: Q - r form
                            float sum = gamma_of(C, h);
#pragma unroll
                            for (int i = 0; i < d; ++i) sum += r[i];
                            static_for<0, d>([&](auto Ii) {
                                constexpr int i = decltype(Ii)::value;
                                constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                                m[slot] = fperm(vn_lane(C, i), satf<FMT>(sum - r[i]));
                            });
                            Q = sum;
                        } else {
                            int sum = gamma_of(C, h);
#pragma unroll
                            for (int i = 0; i < d; ++i) sum += r[i];
                            if constexpr (REG) {
                                static_for<0, d>([&](auto Ii) {
                                    constexpr int i = decltype(Ii)::value;
                                    constexpr int slot = S::T.col_R[C][i] * DC + S::T.col_j[C][i];
                                    m[slot] = (acc_t)__builtin_amdgcn_ds_permute(vn_lane(C, i), sat<FMT>(sum - (int)r[i]));
                                });
                            } else {
#pragma unroll
                                for (int i = 0; i < d; ++i) msg[idx[i]] = (msg_t)sat<FMT>(sum - r[i]);
                            }
                            Q = sum;
                        }
                    } else if constexpr (REG) {
                        Q = Qv[C];
                    } else {
                        Q = (acc_t)Qs[C * ROW + lane + 64 * h];
                    }
                    if constexpr (POST) Qr[C * H + h] = Q;
                    const bool e = Q < (acc_t)0;
                    eb[h] |= (uint64_t)e << C;
                    mask[h] = ballot(e);
                }
                // syndrome accumulation in scalar registers
                static_for<0, d>([&](auto Ii) {
                    constexpr int i = decltype(Ii)::value;
                    constexpr int R = S::T.col_R[C][i];
                    constexpr int slot = R * DC + S::T.col_j[C][i];
                    if constexpr (REG) {
                        // rotate right by s: (m >> s) | (m << c) within each segment
                        const uint32_t s = (uint32_t)cpb->colrot[C][i].s, c = (uint32_t)cpb->colrot[C][i].c;
                        if constexpr (L == 64) {
                            acc[R][0] ^= (mask[0] >> s) | (mask[0] << c);
                        } else {
                            const uint64_t low = cpb->colrot[C][i].low;
                            acc[R][0] ^= ((mask[0] >> s) & low) | ((mask[0] << c) & ~low);
                        }
                    } else if constexpr (GRP) {
                        const uint32_t s = shift_of(slot);
                        const uint64_t low = code->lowmask[slot];
#pragma unroll
                        for (int h = 0; h < H; ++h) acc[R][h] ^= seg_rotr<L>(mask[h], s, low);
                    } else {
                        const uint32_t s = shift_of(slot);
                        uint64_t lo, hi;
                        rotr128(mask[0], mask[H - 1], s, lo, hi);
                        acc[R][0] ^= lo;
                        acc[R][H - 1] ^= hi;
                    }
                });
            });
            if constexpr (REG) {
                if constexpr (RegKnobs::sched_group > 0)
                    if ((decltype(Bc)::value + 1) % RegKnobs::sched_group == 0) __builtin_amdgcn_sched_barrier(0);
            } else {
                sched_group_end<FMT>(decltype(Bc)::value);
            }
        });

        // ---------------- stopping rule, outputs ------------------------------
        uint64_t uns[H];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            uns[h] = 0;
#pragma unroll
            for (int R = 0; R < MB; ++R) uns[h] |= acc[R][h];
        }
        bool conv_now[NG], emit_me[NG];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            bool unsat;
            if constexpr (L < 64) unsat = ((uns[q] >> (g * L)) & G::SEGMASK) != 0;
            else if constexpr (L == 64) unsat = uns[q] != 0;
            else unsat = (uns[0] | uns[H - 1]) != 0;
            conv_now[q] = !unsat;
            emit_me[q] = !done[q] && ((a.early_stop && conv_now[q]) || k == a.max_iters);
            any = any || emit_me[q];
        }
        if (ballot(any)) {
#pragma unroll
            for (int q = 0; q < NG; ++q) {
                if (!ballot(emit_me[q])) continue;
                // stage the packed decisions of group q's shots in LDS
                uint32_t *eq = ebuf + q * (G::SPW * G::EW);
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int C = 0; C < NB; ++C) {
                    if constexpr (GRP) {
                        const uint64_t m = ballot(((eb[q] >> C) & 1ull) != 0);
                        if constexpr (L == 16) {
                            if (lane < 4)
                                reinterpret_cast<uint16_t *>(eq)[lane * G::EW * 2 + C] = (uint16_t)(m >> (16 * lane));
                        } else if constexpr (L == 32) {
                            if (lane < 2) eq[lane * G::EW + C] = (uint32_t)(m >> (32 * lane));
                        } else {
                            if (lane < 2) eq[2 * C + lane] = (uint32_t)(m >> (32 * lane));
                        }
                    } else {
#pragma unroll
                        for (int h = 0; h < H; ++h) {
                            const uint64_t m = ballot(((eb[h] >> C) & 1ull) != 0);
                            if (lane < 2) eq[4 * C + 2 * h + lane] = (uint32_t)(m >> (32 * lane));
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (emit_me[q]) {
                    const long shot = ref[q].shot;
                    for (int w = p; w < G::EW; w += G::SEG) ref[q].err[w] = eq[g * G::EW + w];
                    if (p == 0) {
                        a.conv[shot] = conv_now[q] ? 1 : 0;
                        if (a.iters) a.iters[shot] = (uint8_t)k;
                    }
                    if constexpr (POST) {
#pragma unroll
                        for (int C = 0; C < NB; ++C)
#pragma unroll
                            for (int h = 0; h < H; ++h) {
                                if (grp(h) != q) continue;
                                float qv;
                                if constexpr (FMT == 0) qv = Qr[C * H + h];
                                else qv = (float)Qr[C * H + h] * Fmt<FMT>::post_scale;
                                a.post[shot * G::N + C * L + p + posoff(h)] = qv;
                            }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        bool alldone = true;
#pragma unroll
        for (int q = 0; q < NG; ++q) {
            done[q] = done[q] || emit_me[q];
            alldone = alldone && done[q];
        }
        if (ballot(!alldone) == 0) break;
    }
}

// Waves per SIMD the register allocation must leave room for: as many as
// the kernel's LDS footprint lets a compute unit hold (160 KB / 4 SIMDs),
// capped per format so the scheduler keeps registers for latency hiding.
template <class S, int L, int FMT, int SCHED>
constexpr int wave_occupancy() {
    constexpr size_t b = WaveLds<S, L, FMT, SCHED, 1>::bytes;
    constexpr int per_cu = (int)((160 * 1024) / b);
    constexpr int per_simd = per_cu / 4;
    constexpr int cap = Knobs<FMT>::wave_cap;
    return per_simd < 1 ? 1 : (per_simd > cap ? cap : per_simd);
}

// Workgroups go to the 8 XCDs of the chip in turn (workgroup b to XCD
// b mod 8), each XCD with its own L2.  Giving every XCD one contiguous range
// of wave indices puts neighbouring shots, which share cache lines of the
// packed syndromes and error words, behind one L2.  A bijection of [0, G)
// for any grid size G.
__device__ __forceinline__ long xcd_wave_index(long b, long G) {
    constexpr long X = 8;
    const long q = G / X, r = G % X, x = b % X;
    return x * q + (x < r ? x : r) + b / X;
}

// One wave per workgroup; grid = ceil(batch / shots-per-wave).
template <class S, int L, int FMT, int SCHED, bool PER_BIT, bool POST, int WEIGHTED = 0>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(wave_occupancy<S, L, FMT, SCHED>())))
void k_wave(const DecodeArgs a) {
    using G = Geo<S, L>;
    using Lay = WaveLds<S, L, FMT, SCHED, 1>;
    __shared__ __attribute__((aligned(16))) unsigned char lds[Lay::bytes];
    const int g = (threadIdx.x & 63) / G::SEG;
    const long shot = xcd_wave_index(blockIdx.x, gridDim.x) * G::SPW + g;
    ShotRef ref[1];
    ref[0].shot = shot < a.batch ? shot : -1;
    ref[0].syn = a.syn + (shot < a.batch ? shot : 0) * G::SW;
    ref[0].err = a.err + (shot < a.batch ? shot : 0) * G::EW;
    wave_decode<S, L, FMT, SCHED, PER_BIT, POST, WEIGHTED, 1>(a, a.code, ref, lds);
}

// Register-resident FP32 flooding (L <= 64): LDS holds only the decision
// staging, so occupancy is set by registers.  With per-shot priors and no
// posterior output the working set beside the 120 message registers fits
// three waves per SIMD (168 VGPRs; the only spills are outside the iteration
// loop; with per-edge weights a few reloads per iteration, still faster than
// two waves); per-bit priors or posteriors need two (256 VGPRs).
template <bool PER_BIT, bool POST, int WEIGHTED, int SCHED = 0>
constexpr int reg_waves() { return (!PER_BIT && !POST) ? 3 : 2; }

template <class S, int L, bool PER_BIT, bool POST, int WEIGHTED = 0, int SCHED = 0, int FMT = 0>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(reg_waves<PER_BIT, POST, WEIGHTED, SCHED>())))
void k_wreg(const DecodeArgs a) {
    using G = Geo<S, L>;
    using Lay = WaveLds<S, L, FMT, SCHED, 1, true>;
    __shared__ __attribute__((aligned(16))) unsigned char lds[Lay::bytes];
    const int g = (threadIdx.x & 63) / G::SEG;
    const long shot = xcd_wave_index(blockIdx.x, gridDim.x) * G::SPW + g;
    ShotRef ref[1];
    ref[0].shot = shot < a.batch ? shot : -1;
    ref[0].syn = a.syn + (shot < a.batch ? shot : 0) * G::SW;
    ref[0].err = a.err + (shot < a.batch ? shot : 0) * G::EW;
    wave_decode<S, L, FMT, SCHED, PER_BIT, POST, WEIGHTED, 1, true>(a, a.code, ref, lds);
}

// Neural min-sum inference (per-edge weights, per-shot priors, no posterior).
template <class S, int L>
hipError_t launch_wreg_weighted(const DecodeArgs &a, hipStream_t st) {
    using G = Geo<S, L>;
    const unsigned grid = (unsigned)((a.batch + G::SPW - 1) / G::SPW);
    if (a.weight_iters < a.max_iters)   // neural, then plain iterations
        hipLaunchKernelGGL((k_wreg<S, L, false, false, 2>), dim3(grid), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((k_wreg<S, L, false, false, 1>), dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

template <class S, int L, int SCHED, int FMT>
void launch_wreg_sched(const LaunchKey &k, const DecodeArgs &a, unsigned grid, hipStream_t st) {
    if (k.per_bit) {
        if (k.post) hipLaunchKernelGGL((k_wreg<S, L, true, true, false, SCHED, FMT>), dim3(grid), dim3(64), 0, st, a);
        else hipLaunchKernelGGL((k_wreg<S, L, true, false, false, SCHED, FMT>), dim3(grid), dim3(64), 0, st, a);
    } else {
        if (k.post) hipLaunchKernelGGL((k_wreg<S, L, false, true, false, SCHED, FMT>), dim3(grid), dim3(64), 0, st, a);
        else hipLaunchKernelGGL((k_wreg<S, L, false, false, false, SCHED, FMT>), dim3(grid), dim3(64), 0, st, a);
    }
}

template <class S, int L>
hipError_t launch_wreg(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    using G = Geo<S, L>;
    const unsigned grid = (unsigned)((a.batch + G::SPW - 1) / G::SPW);
    if (k.fmt == 0 && k.sched == 0) launch_wreg_sched<S, L, 0, 0>(k, a, grid, st);
    else if (k.fmt == 0 && k.sched == 1) launch_wreg_sched<S, L, 1, 0>(k, a, grid, st);
    else if (k.fmt == 1 && k.sched == 0) launch_wreg_sched<S, L, 0, 1>(k, a, grid, st);
    else if (k.fmt == 1 && k.sched == 1) launch_wreg_sched<S, L, 1, 1>(k, a, grid, st);
    else return hipErrorNotSupported;
    return hipGetLastError();
}

// int16 messages (FMT = 2), both schedules; instantiated in files of their
// own so that they compile in parallel with the FP32 and int8 kernels.
template <class S, int L>
hipError_t launch_wreg_i16(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    using G = Geo<S, L>;
    const unsigned grid = (unsigned)((a.batch + G::SPW - 1) / G::SPW);
    if (k.fmt != 2) return hipErrorNotSupported;
    if (k.sched == 0) launch_wreg_sched<S, L, 0, 2>(k, a, grid, st);
    else if (k.sched == 1) launch_wreg_sched<S, L, 1, 2>(k, a, grid, st);
    else return hipErrorNotSupported;
    return hipGetLastError();
}

template <class S, int L, int FMT, int SCHED, bool PB, bool PO>
hipError_t launch_wave_one(const DecodeArgs &a, hipStream_t st) {
    using G = Geo<S, L>;
    const unsigned grid = (unsigned)((a.batch + G::SPW - 1) / G::SPW);
    hipLaunchKernelGGL((k_wave<S, L, FMT, SCHED, PB, PO>), dim3(grid), dim3(64), 0, st, a);
    return hipGetLastError();
}

template <class S, int L, int FMT, int SCHED>
hipError_t launch_wave(const LaunchKey &k, const DecodeArgs &a, hipStream_t st) {
    if (k.per_bit)
        return k.post ? launch_wave_one<S, L, FMT, SCHED, true, true>(a, st)
                      : launch_wave_one<S, L, FMT, SCHED, true, false>(a, st);
    return k.post ? launch_wave_one<S, L, FMT, SCHED, false, true>(a, st)
                  : launch_wave_one<S, L, FMT, SCHED, false, false>(a, st);
}

}  // namespace qldpc
