// Mixed-code persistent decoding: one launch sequence decodes a batch whose
// shots belong to different lifted codes (L in {16, 32, 64, 128}) with their
// own priors (Section 2, Algorithm 1 per shot; batching as the paper's
// asynchronous multi-decoder proposal, Table 1).
//
// Shots are bucketed by code on the device (counting pass, then a scatter
// into a code-ordered index list, largest L first).  One persistent grid of
// wavefronts per (block pattern, lift size) then claims tiles of same-code
// shots from its own atomic counter until none are left: for L <= 64 every
// message stays in registers (one 64-lane group of 64 / L shots per tile),
// for L = 128 in the LDS of a persistent workgroup of 8 waves running the
// workgroup-per-shot decoder (one shot per tile).  Codes of both patterns (H_Z and
// H_X of one CSS code, say) can share a batch, so both sides of a code are
// decoded in one launch sequence.  Each shot's result depends only on its
// own syndrome and prior, never on its tile mates or grid.
#pragma once
#include "decode_block.h"
#include "decode_wave.h"

namespace qldpc {

constexpr int kMaxMixCodes = 8;
constexpr int kMixBlockWaves = 8;   // waves per workgroup of the L = 128 grid

struct MixedArgs {
    DecodeArgs base;                       // alpha, iterations, priors, conv / iters outputs
    const DevCode *codes[kMaxMixCodes];
    int32_t L[kMaxMixCodes];
    int32_t which[kMaxMixCodes];           // block pattern: 0 = H_Z, 1 = H_X
    int32_t rank[kMaxMixCodes];            // bucket order of each code (largest L first)
    int32_t ncodes;
    const int32_t *shot_code;              // [batch]
    const int64_t *syn_off;                // [batch], words into syn
    const int64_t *err_off;                // [batch], words into err
    const uint32_t *syn;
    uint32_t *err;
    int32_t *scratch;                      // counts[8], cursors[8], tile counters[8], order[batch]
    int32_t batch;
};

namespace mix {

__device__ __forceinline__ int32_t *counts(const MixedArgs &m) { return m.scratch; }
__device__ __forceinline__ int32_t *cursors(const MixedArgs &m) { return m.scratch + kMaxMixCodes; }
constexpr int kMixGrids = 8;   // one persistent grid per (pattern, lift size 16 / 32 / 64 / 128)
constexpr int kScratchHead = 2 * kMaxMixCodes + kMixGrids;

__host__ __device__ __forceinline__ int grid_of(int which, int L) {
    return 4 * which + (L == 16 ? 0 : L == 32 ? 1 : L == 64 ? 2 : 3);
}
__device__ __forceinline__ int32_t *tile_ctr(const MixedArgs &m, int which, int L) {
    return m.scratch + 2 * kMaxMixCodes + grid_of(which, L);
}
__device__ __forceinline__ int32_t *order(const MixedArgs &m) { return m.scratch + kScratchHead; }
__host__ __device__ constexpr int shots_per_tile(int L) { return L <= 64 ? 64 / L : 1; }

}  // namespace mix

__global__ void k_mix_clear(const MixedArgs m) {
    if (threadIdx.x < mix::kScratchHead) m.scratch[threadIdx.x] = 0;
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
    constexpr bool REG = L <= 64;
    const int g = (threadIdx.x & 63) / G::SEG;
    ShotRef ref[1];
    long shot = g < cnt ? (long)mix::order(m)[first + g] : -1;
    int64_t so = shot >= 0 ? m.syn_off[shot] : 0, eo = shot >= 0 ? m.err_off[shot] : 0;
    if constexpr (G::SPW == 1) {
        // one shot per wave: keep its index and offsets in scalar registers
        shot = (long)(int64_t)wave::uniform64((uint64_t)shot);
        so = (int64_t)wave::uniform64((uint64_t)so);
        eo = (int64_t)wave::uniform64((uint64_t)eo);
    }
    ref[0].shot = shot;
    ref[0].syn = m.syn + so;
    ref[0].err = m.err + eo;
    wave_decode<S, L, 0, 0, false, false, false, 1, REG>(m.base, m.codes[c], ref, lds);
}

// Persistent decoder of the shots whose code has pattern S and lift size L.  A claimed
// tile is located by a short scalar walk over the codes in bucket order, so
// nothing but pointers stays live across tiles (the decoder body needs the
// registers).  Waves per SIMD: three for L <= 32; two for L = 64, whose
// body inside the persistent loop would spill within the iteration loop at
// three (two measured 4 % faster); one 61 KB LDS wave for L = 128.
template <class S, int L>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(L <= 32 ? 3 : L == 64 ? 2 : 1)))
void k_mix_decode(const MixedArgs m) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[WaveLds<S, L, 0, 0, 1, (L <= 64)>::bytes];
    constexpr int spt = mix::shots_per_tile(L);
    for (;;) {
        int t = 0;
        if ((threadIdx.x & 63) == 0) t = atomicAdd(mix::tile_ctr(m, S::WHICH, L), 1);
        t = __builtin_amdgcn_readfirstlane(t);
        int c = -1, first = 0, cnt = 0;
        for (int r = 0, acc = 0, tiles = 0; r < m.ncodes; ++r) {
            int cc = 0;
            for (int d = 0; d < m.ncodes; ++d)
                if (m.rank[d] == r) cc = d;
            const int n = __builtin_amdgcn_readfirstlane(mix::counts(m)[cc]);
            if (m.L[cc] == L && m.which[cc] == S::WHICH) {
                const int nt = (n + spt - 1) / spt;
                if (c < 0 && t < tiles + nt) {
                    c = cc;
                    first = acc + (t - tiles) * spt;
                    cnt = min(spt, n - (t - tiles) * spt);
                }
                tiles += nt;
            }
            acc += n;
        }
        if (c < 0) return;   // every tile of this pattern and lift size is taken
        mix_tile<S, L>(m, c, first, cnt, lds);
    }
}

// Locates tile t of the codes with pattern S::WHICH and lift L (spt shots
// per tile) by a scalar walk over the bucket order: code c, first index into
// the order list, shot count; c = -1 once t is past the last tile.
template <class S, int L, int spt>
__device__ __forceinline__ void mix_locate(const MixedArgs &m, int t, int &c, int &first, int &cnt) {
    c = -1;
    first = cnt = 0;
    for (int r = 0, acc = 0, tiles = 0; r < m.ncodes; ++r) {
        int cc = 0;
        for (int d = 0; d < m.ncodes; ++d)
            if (m.rank[d] == r) cc = d;
        const int n = __builtin_amdgcn_readfirstlane(mix::counts(m)[cc]);
        if (m.L[cc] == L && m.which[cc] == S::WHICH) {
            const int nt = (n + spt - 1) / spt;
            if (c < 0 && t < tiles + nt) {
                c = cc;
                first = acc + (t - tiles) * spt;
                cnt = min(spt, n - (t - tiles) * spt);
            }
            tiles += nt;
        }
        acc += n;
    }
}

// Persistent decoder of the L = 128 shots: each 8-wave workgroup claims one
// shot at a time and decodes it with its messages in LDS (61 KB FP32, two
// workgroups per compute unit).  Every value that decides whether a wave
// reaches a barrier is workgroup-uniform (broadcast through LDS, then
// readfirstlane).
template <class S>
__global__ __launch_bounds__(64 * kMixBlockWaves) void k_mix_block(const MixedArgs m) {
    constexpr int L = 128, NW = kMixBlockWaves;
    __shared__ __attribute__((aligned(16))) unsigned char lds[BlockLds<S, L, 0, NW>::bytes];
    __shared__ int tile;
    for (;;) {
        if (threadIdx.x == 0) tile = atomicAdd(mix::tile_ctr(m, S::WHICH, L), 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(tile);
        __syncthreads();   // everyone has read tile before it is claimed again
        int c, first, cnt;
        mix_locate<S, L, 1>(m, t, c, first, cnt);
        if (c < 0) return;   // every L = 128 tile of this pattern is taken
        const long shot = (long)(int64_t)wave::uniform64((uint64_t)(int64_t)mix::order(m)[first]);
        const int64_t so = (int64_t)wave::uniform64((uint64_t)m.syn_off[shot]);
        const int64_t eo = (int64_t)wave::uniform64((uint64_t)m.err_off[shot]);
        block_decode<S, L, 0, NW, false, false>(m.base, m.codes[c], shot, m.syn + so, m.err + eo, lds);
        __syncthreads();   // LDS reused by the next shot
    }
}

}  // namespace qldpc
