// gv_compact.h -- stable three-way compaction of track outputs into the
// per-particle-type queues (the stage baskets and survivor stack of
// Sec. 2.1.1-2.1.2, realised as queues in HBM).
//
// Every input slot expands to at most three outputs (the surviving track and
// two secondaries), each bound for one of three queues.  Output order in a
// queue is the order of the expanded input stream: input slot, then
// (survivor, child 0, child 1).  One pass, no atomics deciding order:
//   1. per wave: ballot + popcount of the two bits of each thread's per-queue
//      count (0..3) gives the wave-exclusive offset and the wave total;
//   2. per block: wave totals through LDS;
//   3. across blocks: single-pass decoupled look-back over the chunk index
//      (chunks are claimed in increasing order, so every predecessor is owned
//      by a resident workgroup); status words carry an epoch so they never
//      need clearing between launches.
#pragma once
#include "gv_common.h"

namespace gv {

// status word: [epoch:30 | flag:2 | value:32]; flag 1 = aggregate, 2 = inclusive prefix
constexpr uint64_t kFlagAgg = 1ull, kFlagInc = 2ull;
__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint64_t flag, uint32_t v)
{
    return ((uint64_t)epoch << 34) | (flag << 32) | v;
}

template <int BLOCK> struct ScanShared {
    int wtot[3][BLOCK / 64];
    int prefix[3];
    int total[3];
    int ticket;
};

// exclusive offsets of this thread's counts within the block, and block totals
template <int BLOCK>
__device__ __forceinline__ void block_scan3(const int cnt[3], int excl[3], int tot[3], ScanShared<BLOCK>& sh)
{
    constexpr int NW = BLOCK / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int wex[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const uint64_t b0 = __ballot(cnt[q] & 1), b1 = __ballot(cnt[q] & 2);
        wex[q] = __popcll(b0 & lt) + 2 * __popcll(b1 & lt);
        if (lane == 0) sh.wtot[q][wid] = __popcll(b0) + 2 * __popcll(b1);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        int before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int v = sh.wtot[q][w];
            before += w < wid ? v : 0;
            all += v;
        }
        excl[q] = before + wex[q];
        tot[q] = all;
    }
}

// Publish this chunk's aggregates, look back for the exclusive prefix of each
// queue, publish the inclusive prefix.  Called by all threads; lanes 0..2 of
// wave 0 do the work; the result lands in sh.prefix.
template <int BLOCK>
__device__ __forceinline__ void lookback3(uint64_t* status, uint32_t chunk, uint32_t epoch, const int tot[3],
                                          ScanShared<BLOCK>& sh)
{
    const int q = threadIdx.x;
    if (q < 3) {
        uint64_t* my = status + (size_t)chunk * 3 + q;
        uint32_t excl = 0;
        if (chunk == 0) {
            __hip_atomic_store(my, pack_status(epoch, kFlagInc, (uint32_t)tot[q]), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(my, pack_status(epoch, kFlagAgg, (uint32_t)tot[q]), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
            long long j = (long long)chunk - 1;
            while (j >= 0) {
                const uint64_t s = __hip_atomic_load(status + (size_t)j * 3 + q, __ATOMIC_ACQUIRE,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t ep = (uint32_t)(s >> 34);
                const uint64_t fl = (s >> 32) & 3ull;
                if (ep != epoch || fl == 0) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += (uint32_t)s;
                if (fl == kFlagInc) break;
                --j;
            }
            __hip_atomic_store(my, pack_status(epoch, kFlagInc, excl + (uint32_t)tot[q]), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        sh.prefix[q] = (int)excl;
        sh.total[q] = tot[q];
    }
    __syncthreads();
}

}  // namespace gv
