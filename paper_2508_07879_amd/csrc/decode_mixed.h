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
// for L = 128 in the registers of a persistent workgroup of two waves, each
// holding half of every circulant's rows (one shot per tile).  Codes of both
// patterns (H_Z and H_X of one CSS code, say) can share a batch, so both sides of a code are
// decoded in one launch sequence.  Each shot's result depends only on its
// own syndrome and prior, never on its tile mates or grid.
#pragma once
#include "decode_wave.h"
#include "decode_wreg2.h"

namespace qldpc {

constexpr int kMaxMixCodes = 8;

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
    int32_t *scratch;                      // see the mix:: accessors; then order[batch]
    int32_t batch;
};

namespace mix {

constexpr int kMixGrids = 8;   // one persistent grid per (pattern, lift size 16 / 32 / 64 / 128)

// Per-grid tile table, written by k_mix_plan: the codes of the grid in bucket
// order, each with its first index into the order list, its shot count and
// the running tile count at its end.
struct GridEntry {
    int32_t code, first, count, tiles_end;
};

// Scratch head (int32 words): counts[8] | cursors[8] | tile counters[8] |
// order offset per code[8] | entries per grid[8] | grid tables[8][8] |
// device code table pointers[8]; then the order list.
constexpr int kCounts = 0, kCursors = 8, kTiles = 16, kOffs = 24, kNEnt = 32, kEnt = 40;
constexpr int kCodePtr = kEnt + kMixGrids * kMaxMixCodes * 4;       // 8-byte aligned (296)
constexpr int kScratchHead = kCodePtr + 2 * kMaxMixCodes;

__device__ __forceinline__ int32_t *counts(const MixedArgs &m) { return m.scratch + kCounts; }
__device__ __forceinline__ int32_t *cursors(const MixedArgs &m) { return m.scratch + kCursors; }
__device__ __forceinline__ int32_t *offs(const MixedArgs &m) { return m.scratch + kOffs; }
__device__ __forceinline__ int32_t *n_entries(const MixedArgs &m) { return m.scratch + kNEnt; }
__device__ __forceinline__ GridEntry *entries(const MixedArgs &m, int g) {
    return reinterpret_cast<GridEntry *>(m.scratch + kEnt) + g * kMaxMixCodes;
}
__device__ __forceinline__ const DevCode **code_table(const MixedArgs &m) {
    return reinterpret_cast<const DevCode **>(m.scratch + kCodePtr);
}

__host__ __device__ __forceinline__ int grid_of(int which, int L) {
    return 4 * which + (L == 16 ? 0 : L == 32 ? 1 : L == 64 ? 2 : 3);
}
__device__ __forceinline__ int32_t *tile_ctr(const MixedArgs &m, int which, int L) {
    return m.scratch + kTiles + grid_of(which, L);
}
__device__ __forceinline__ int32_t *order(const MixedArgs &m) { return m.scratch + kScratchHead; }
__host__ __device__ constexpr int shots_per_tile(int L) { return L <= 64 ? 64 / L : 1; }

// Locates tile t of grid g (spt shots per tile) in the grid's table: the
// code, the first index into the order list, the shot count; c = -1 once t
// is past the last tile.  Reads the table from device memory each time (the
// persistent loops call it after claiming a tile with an atomic, so nothing
// of it stays in scalar registers across a decode).
__device__ __forceinline__ void locate(const MixedArgs &m, int g, int spt, int t, int &c, int &first, int &cnt) {
    c = -1;
    first = cnt = 0;
    const int ne = __builtin_amdgcn_readfirstlane(n_entries(m)[g]);
    const GridEntry *E = entries(m, g);
    int start = 0;
    for (int k = 0; k < ne; ++k) {
        const int end = __builtin_amdgcn_readfirstlane(E[k].tiles_end);
        if (t < end) {
            c = __builtin_amdgcn_readfirstlane(E[k].code);
            const int n = __builtin_amdgcn_readfirstlane(E[k].count);
            first = __builtin_amdgcn_readfirstlane(E[k].first) + (t - start) * spt;
            cnt = min(spt, n - (t - start) * spt);
            return;
        }
        start = end;
    }
}

}  // namespace mix

__global__ void k_mix_clear(const MixedArgs m) {
    const int i = threadIdx.x;
    if (i < mix::kOffs) m.scratch[i] = 0;                    // counts, cursors, tile counters
    if (i < kMaxMixCodes) mix::code_table(m)[i] = i < m.ncodes ? m.codes[i] : nullptr;
}

// Counts shots per code: a workgroup histogram in LDS over a grid-stride
// range of shots, then one global atomic per code per workgroup.
constexpr int kBucketThreads = 1024;

__global__ __launch_bounds__(kBucketThreads) void k_mix_count(const MixedArgs m) {
    __shared__ int h[kMaxMixCodes];
    if (threadIdx.x < kMaxMixCodes) h[threadIdx.x] = 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m.batch; i += gridDim.x * blockDim.x) {
        const int c = m.shot_code[i];
        if (c >= 0 && c < m.ncodes) atomicAdd(&h[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxMixCodes && h[threadIdx.x] > 0) atomicAdd(&mix::counts(m)[threadIdx.x], h[threadIdx.x]);
}

// Order offsets per code (codes in bucket order: largest L first) and the
// per-grid tile tables.  One wave.
__global__ void k_mix_plan(const MixedArgs m) {
    if (threadIdx.x != 0) return;
    int tiles[mix::kMixGrids] = {}, ne[mix::kMixGrids] = {};
    for (int r = 0, acc = 0; r < m.ncodes; ++r) {
        int cc = 0;
        for (int d = 0; d < m.ncodes; ++d)
            if (m.rank[d] == r) cc = d;
        const int n = mix::counts(m)[cc];
        mix::offs(m)[cc] = acc;
        const int g = mix::grid_of(m.which[cc], m.L[cc]);
        const int spt = mix::shots_per_tile(m.L[cc]);
        tiles[g] += (n + spt - 1) / spt;
        mix::entries(m, g)[ne[g]++] = mix::GridEntry{cc, acc, n, tiles[g]};
        acc += n;
    }
    for (int g = 0; g < mix::kMixGrids; ++g) mix::n_entries(m)[g] = ne[g];
}

// Scatters shot indices into the code-ordered list.  Each workgroup takes
// the same grid-stride range as in k_mix_count: it counts its shots per code
// in LDS, reserves one block of positions per code with one global atomic,
// then places every shot at its code's offset + the block base + a rank from
// an LDS counter.  (The order of shots within a code is immaterial: every
// shot's result depends only on its own inputs.)
__global__ __launch_bounds__(kBucketThreads) void k_mix_scatter(const MixedArgs m) {
    __shared__ int h[kMaxMixCodes], base[kMaxMixCodes], cur[kMaxMixCodes];
    if (threadIdx.x < kMaxMixCodes) h[threadIdx.x] = cur[threadIdx.x] = 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m.batch; i += gridDim.x * blockDim.x) {
        const int c = m.shot_code[i];
        if (c >= 0 && c < m.ncodes) atomicAdd(&h[c], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxMixCodes)
        base[threadIdx.x] = h[threadIdx.x] > 0 ? atomicAdd(&mix::cursors(m)[threadIdx.x], h[threadIdx.x]) : 0;
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m.batch; i += gridDim.x * blockDim.x) {
        const int c = m.shot_code[i];
        if (c >= 0 && c < m.ncodes) mix::order(m)[mix::offs(m)[c] + base[c] + atomicAdd(&cur[c], 1)] = i;
    }
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
    const DevCode *code = (const DevCode *)wave::uniform64((uint64_t)mix::code_table(m)[c]);
    wave_decode<S, L, 0, 0, false, false, false, 1, REG>(m.base, code, ref, lds);
}

// Persistent decoder of the shots whose code has pattern S and lift size L.
// A claimed tile is located in the grid's table in device memory, so nothing
// but pointers stays live across tiles (the decoder body needs the
// registers).  Three waves per SIMD for L <= 64 (messages in registers), one
// 61 KB LDS wave for L = 128.
template <class S, int L>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(L <= 64 ? 3 : 1)))
void k_mix_decode(const MixedArgs m) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[WaveLds<S, L, 0, 0, 1, (L <= 64)>::bytes];
    constexpr int spt = mix::shots_per_tile(L);
    for (;;) {
        int t = 0;
        if ((threadIdx.x & 63) == 0) t = atomicAdd(mix::tile_ctr(m, S::WHICH, L), 1);
        t = __builtin_amdgcn_readfirstlane(t);
        int c, first, cnt;
        mix::locate(m, mix::grid_of(S::WHICH, L), spt, t, c, first, cnt);
        if (c < 0) return;   // every tile of this pattern and lift size is taken
        mix_tile<S, L>(m, c, first, cnt, lds);
    }
}

// Persistent decoder of the L = 128 shots: each workgroup of two waves claims
// one shot at a time and decodes it with its messages in registers (three
// waves per SIMD, six workgroups per compute unit).  Every value that decides
// whether a wave reaches a barrier is workgroup-uniform (broadcast through
// LDS, then readfirstlane).
template <class S>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_mix_wreg2(const MixedArgs m) {
    __shared__ wreg2::Lds<S, 0, 128> sh;
    __shared__ int tile;
    for (;;) {
        if (threadIdx.x == 0) tile = atomicAdd(mix::tile_ctr(m, S::WHICH, 128), 1);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(tile);
        __syncthreads();   // both waves have read tile before it is claimed again
        int c, first, cnt;
        mix::locate(m, mix::grid_of(S::WHICH, 128), 1, t, c, first, cnt);
        if (c < 0) return;   // every L = 128 tile of this pattern is taken
        const long shot = (long)(int64_t)wave::uniform64((uint64_t)(int64_t)mix::order(m)[first]);
        const int64_t so = (int64_t)wave::uniform64((uint64_t)m.syn_off[shot]);
        const int64_t eo = (int64_t)wave::uniform64((uint64_t)m.err_off[shot]);
        const DevCode *code = (const DevCode *)wave::uniform64((uint64_t)mix::code_table(m)[c]);
        wreg2_decode<S, 0, false, false, 128>(m.base, code, shot, m.syn + so, m.err + eo, sh);
        __syncthreads();   // LDS reused by the next shot
    }
}

}  // namespace qldpc
