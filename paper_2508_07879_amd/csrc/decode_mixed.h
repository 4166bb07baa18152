// Mixed-code persistent decoding: one launch decodes a batch whose shots
// belong to different lifted codes (L in {16, 32, 64, 128}) with their own
// priors (Section 2, Algorithm 1 per shot; batching as the paper's
// asynchronous multi-decoder proposal, Table 1).
//
// Shots are bucketed by code on the device (counting pass, then a scatter
// into a code-ordered index list, largest L first).  A persistent grid of
// wavefronts then claims tiles of same-code shots from an atomic counter
// until none are left.  Every wave reserves the LDS of one L = 128 shot
// (61 KB); an L <= 64 tile uses it as two independent 64-lane groups, i.e.
// 2 * 64 / L shots per tile.  Each shot's result depends only on its own
// syndrome and prior, never on its tile mates.
#pragma once
#include "decode_wave.h"

namespace qldpc {

constexpr int kMaxMixCodes = 8;

struct MixedArgs {
    DecodeArgs base;                       // alpha, iterations, priors, conv / iters outputs
    const DevCode *codes[kMaxMixCodes];
    int32_t L[kMaxMixCodes];
    int32_t rank[kMaxMixCodes];            // bucket order of each code (largest L first)
    int32_t ncodes;
    const int32_t *shot_code;              // [batch]
    const int64_t *syn_off;                // [batch], words into syn
    const int64_t *err_off;                // [batch], words into err
    const uint32_t *syn;
    uint32_t *err;
    int32_t *scratch;                      // counts[8], cursors[8], tile counter, order[batch]
    int32_t batch;
};

namespace mix {

__device__ __forceinline__ int32_t *counts(const MixedArgs &m) { return m.scratch; }
__device__ __forceinline__ int32_t *cursors(const MixedArgs &m) { return m.scratch + kMaxMixCodes; }
__device__ __forceinline__ int32_t *tile_ctr(const MixedArgs &m) { return m.scratch + 2 * kMaxMixCodes; }
__device__ __forceinline__ int32_t *order(const MixedArgs &m) { return m.scratch + 2 * kMaxMixCodes + 1; }

__device__ __forceinline__ int shots_per_tile(int L) { return L <= 64 ? 2 * (64 / L) : 1; }

}  // namespace mix

__global__ void k_mix_clear(const MixedArgs m) {
    if (threadIdx.x <= 2 * kMaxMixCodes) m.scratch[threadIdx.x] = 0;
}

__global__ void k_mix_count(const MixedArgs m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.batch) return;
    const int c = m.shot_code[i];
    if (c >= 0 && c < m.ncodes) atomicAdd(&mix::counts(m)[c], 1);
}

__global__ void k_mix_scatter(const MixedArgs m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.batch) return;
    const int c = m.shot_code[i];
    if (c < 0 || c >= m.ncodes) return;
    int off = 0;
    for (int d = 0; d < m.ncodes; ++d)
        if (m.rank[d] < m.rank[c]) off += mix::counts(m)[d];
    const int pos = off + atomicAdd(&mix::cursors(m)[c], 1);
    mix::order(m)[pos] = i;
}

template <class S, int L>
__device__ __forceinline__ void mix_tile(const MixedArgs &m, int c, int first, int cnt, unsigned char *lds) {
    using G = Geo<S, L>;
    constexpr int NG = L <= 64 ? 2 : 1;
    const int g = (threadIdx.x & 63) / G::SEG;
    ShotRef ref[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        const int j = q * G::SPW + g;
        const long shot = j < cnt ? (long)mix::order(m)[first + j] : -1;
        ref[q].shot = shot;
        ref[q].syn = m.syn + (shot >= 0 ? m.syn_off[shot] : 0);
        ref[q].err = m.err + (shot >= 0 ? m.err_off[shot] : 0);
    }
    wave_decode<S, L, 0, 0, false, false, false, NG>(m.base, m.codes[c], ref, lds);
}

template <class S>
__global__ __launch_bounds__(64) void k_mix_decode(const MixedArgs m) {
    constexpr size_t kLds = WaveLds<S, 128, 0, 0, 1>::bytes > WaveLds<S, 64, 0, 0, 2>::bytes
                                ? WaveLds<S, 128, 0, 0, 1>::bytes
                                : WaveLds<S, 64, 0, 0, 2>::bytes;
    static_assert(WaveLds<S, 16, 0, 0, 2>::bytes <= kLds && WaveLds<S, 32, 0, 0, 2>::bytes <= kLds, "LDS");
    __shared__ __attribute__((aligned(16))) unsigned char lds[kLds];
    // tiles per code, in bucket order
    int ntile[kMaxMixCodes], nshot[kMaxMixCodes], tile0[kMaxMixCodes], shot0[kMaxMixCodes];
    int total = 0;
    for (int r = 0; r < m.ncodes; ++r) {
        int c = 0;
        for (int d = 0; d < m.ncodes; ++d)
            if (m.rank[d] == r) c = d;
        nshot[c] = __builtin_amdgcn_readfirstlane(mix::counts(m)[c]);
        ntile[c] = (nshot[c] + mix::shots_per_tile(m.L[c]) - 1) / mix::shots_per_tile(m.L[c]);
        tile0[c] = total;
        total += ntile[c];
    }
    for (int r = 0, acc = 0; r < m.ncodes; ++r) {
        for (int d = 0; d < m.ncodes; ++d)
            if (m.rank[d] == r) {
                shot0[d] = acc;
                acc += nshot[d];
            }
    }
    for (;;) {
        int t = 0;
        if ((threadIdx.x & 63) == 0) t = atomicAdd(mix::tile_ctr(m), 1);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= total) return;
        int c = 0;
        for (int d = 0; d < m.ncodes; ++d)
            if (t >= tile0[d] && t < tile0[d] + ntile[d]) c = d;
        const int spt = mix::shots_per_tile(m.L[c]);
        const int local = t - tile0[c];
        const int first = shot0[c] + local * spt;
        const int cnt = min(spt, nshot[c] - local * spt);
        switch (m.L[c]) {
            case 16: mix_tile<S, 16>(m, c, first, cnt, lds); break;
            case 32: mix_tile<S, 32>(m, c, first, cnt, lds); break;
            case 64: mix_tile<S, 64>(m, c, first, cnt, lds); break;
            default: mix_tile<S, 128>(m, c, first, cnt, lds); break;
        }
    }
}

}  // namespace qldpc
