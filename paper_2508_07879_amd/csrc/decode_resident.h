// Resident latency decoder: the workgroup-per-shot decoder kept on the GPU
// between requests, so that a request costs neither a kernel launch nor a
// stream synchronisation.
//
// The grid has one workgroup per shot slot.  The whole of wave 0 of
// workgroup 0 polls the doorbell page in mapped host memory (every lane
// loads, so the poll loop and its exit are wave-uniform); on a new sequence
// number it relays [sequence, batch] to the other workgroups through a
// device-memory mailbox.
// Workgroup w < batch decodes shot w from the mapped staging buffers (inputs
// written by the host before it rang), makes its results visible to the
// host, then publishes the sequence number in done_seq[w].
//
// CSS pairs (SX not void): the two sides of one CSS code share the grid;
// even shots are syndromes of the H_Z pattern (table a.code), odd shots of the
// H_X pattern (table code_x), so one request decodes both sides of each of
// its syndrome pairs at once (the paper's unit of latency, Section 2).
//
// Exit: workgroup 0 leaves when the host sets `stop` or when no request has
// arrived for `idle_ticks` of the GPU's constant wall clock, and tells the
// others through the mailbox; they also leave on their own after twice that
// time without word from it, so every wave of the grid ends within a bounded
// time whatever the host does.  The host relaunches a grid that has exited.
#pragma once
#include "decode_block.h"

namespace qldpc {

constexpr uint64_t kResidentExit = ~0ull;

__device__ __forceinline__ uint64_t sys_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

using wave::uniform64;

// Every branch that decides whether a wave reaches a barrier depends only on
// wave-uniform values (scalar registers): the whole of wave 0 polls, and
// what it finds is read back through readfirstlane.  With a branch the
// compiler must treat as divergent (say, "thread 0 polls" followed by a
// barrier in the same loop) it may let the other lanes of the wave run on to
// the next barrier without the polling lane, which then never runs again.
template <class S, int L, int FMT, int NW, bool PER_BIT, class SX = void>
__global__ __launch_bounds__(64 * NW) void k_resident(const ResidentArgs r) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[BlockLds<S, L, FMT, NW>::bytes];
    __shared__ uint64_t req[2];   // [sequence or kResidentExit, batch]
    constexpr int kSW = (S::MB * L + 31) / 32, kEW = (S::NB * L + 31) / 32;
    const int wg = blockIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    uint64_t seen = r.start_seq;
    for (;;) {
        if (wv == 0) {
            uint64_t got = kResidentExit, batch = 0;
            const uint64_t t0 = wall_clock64();
            if (wg == 0) {
                for (;;) {
                    const uint64_t q = uniform64(sys_load(&r.ring->req_seq));
                    if (q != seen) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        got = q;
                        batch = (uint64_t)__builtin_amdgcn_readfirstlane(
                            __hip_atomic_load(&r.ring->batch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
                        break;
                    }
                    if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(&r.ring->stop, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_SYSTEM)) != 0)
                        break;
                    if (wall_clock64() - t0 > r.idle_ticks) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                if (gridDim.x > 1 && lane == 0) {
                    __hip_atomic_store(&r.cmd[1], batch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&r.cmd[0], got, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            } else {
                for (;;) {
                    const uint64_t q =
                        uniform64(__hip_atomic_load(&r.cmd[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                    if (q != seen) {
                        // one system-scope acquire: wave 0's mailbox and, through
                        // workgroup 0's chain, the host's inputs
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        got = q;
                        batch = uniform64(__hip_atomic_load(&r.cmd[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                        break;
                    }
                    if (wall_clock64() - t0 > 2 * r.idle_ticks) break;
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            if (lane == 0) {
                req[0] = got;
                req[1] = batch;
            }
        }
        __syncthreads();
        const uint64_t got = uniform64(req[0]);
        const int batch = (int)__builtin_amdgcn_readfirstlane((uint32_t)req[1]);
        __syncthreads();   // everyone has read req before wave 0 may rewrite it
        if (got == kResidentExit) return;
        seen = got;
        if (wg < batch) {
            // Wave 0 acquired at system scope after it saw the request; the
            // barriers above order the other waves of the workgroup (one
            // compute unit, one L1) after that acquire.
            if constexpr (std::is_void<SX>::value) {
                block_decode<S, L, FMT, NW, PER_BIT, false>(r.a, r.a.code, wg, r.a.syn + wg * kSW,
                                                            r.a.err + wg * kEW, lds);
            } else if (wg & 1) {   // uniform over the workgroup
                block_decode<SX, L, FMT, NW, PER_BIT, false>(r.a, r.code_x, wg, r.a.syn + wg * kSW,
                                                             r.a.err + wg * kEW, lds);
            } else {
                block_decode<S, L, FMT, NW, PER_BIT, false>(r.a, r.a.code, wg, r.a.syn + wg * kSW,
                                                            r.a.err + wg * kEW, lds);
            }
            // Each wave waits until its own result stores have completed, then
            // thread 0 answers with a system-scope release store (one L2
            // write-back per request instead of one per wave).
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_store(&r.ring->done_seq[wg], got, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// Sets the mailbox to "nothing after `seq`" before a grid starts (a kernel
// rather than a memset: the previous grid may have left its exit word there).
static __global__ void k_resident_arm(uint64_t *cmd, uint64_t seq) {
    if (threadIdx.x == 0) {
        cmd[0] = seq;
        cmd[1] = 0;
    }
}

template <class S, int L, int FMT, int NW, class SX = void>
hipError_t launch_resident(const LaunchKey &k, const ResidentArgs &r, int grid, hipStream_t st) {
    if (k.post) return hipErrorNotSupported;
    if constexpr (!std::is_void<SX>::value) {
        static_assert(BlockLds<SX, L, FMT, NW>::bytes == BlockLds<S, L, FMT, NW>::bytes,
                      "the two sides of a pair share one LDS layout");
        if (r.code_x == nullptr || grid % 2 != 0) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_resident_arm, dim3(1), dim3(64), 0, st, r.cmd, r.start_seq);
    if (k.per_bit)
        hipLaunchKernelGGL((k_resident<S, L, FMT, NW, true, SX>), dim3((unsigned)grid), dim3(64 * NW), 0, st, r);
    else
        hipLaunchKernelGGL((k_resident<S, L, FMT, NW, false, SX>), dim3((unsigned)grid), dim3(64 * NW), 0, st, r);
    return hipGetLastError();
}

}  // namespace qldpc
