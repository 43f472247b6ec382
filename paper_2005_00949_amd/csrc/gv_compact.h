// gv_compact.h -- three-way compaction of track outputs into the
// per-particle-type queues (the stage baskets and survivor stack of
// Sec. 2.1.1-2.1.2, realised as queues in HBM): stable across the whole
// launch (look-back) or stable within each block (arrival-order reservation).
//
// Every input slot expands to at most three outputs (the surviving track and
// two secondaries), each bound for one of three queues.  Output order in a
// queue is the order of the expanded input stream: input slot, then
// (survivor, child 0, child 1).  One pass, no atomics deciding order:
//   1. per wave: ballot + popcount of the two bits of each thread's per-queue
//      count (0..3) gives the wave-exclusive offset and the wave total;
//   2. per block: wave totals through LDS;
//   3. across blocks: single-pass decoupled look-back over the chunk index,
//      one wave reading 64 predecessors per round (chunks are claimed in
//      increasing order, so every predecessor is owned by a running
//      workgroup); status words carry an epoch so they never need clearing
//      between launches.
#pragma once
#include "gv_common.h"

namespace gv {

// status word: [epoch:30 | flag:2 | value:32]; flag 1 = aggregate, 2 = inclusive prefix
constexpr uint64_t kFlagAgg = 1ull, kFlagInc = 2ull;
// bound on the polls of one look-back window (each poll sleeps ~64 cycles);
// past it the error flag is raised and the launch completes with a wrong count
constexpr uint32_t kMaxSpins = 1u << 22;
constexpr uint32_t kEpochBits = (1u << 30) - 1u;
__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint64_t flag, uint32_t v)
{
    return ((uint64_t)(epoch & kEpochBits) << 34) | (flag << 32) | v;
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

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off, 64);
    return v;
}

// Exclusive prefix of queue q for `chunk`: wave 0 reads the status words of
// the 64 preceding chunks at once, finds the nearest inclusive prefix by
// ballot and adds the aggregates up to it; a window without an inclusive
// prefix is summed whole and the window moves 64 chunks back.
__device__ __forceinline__ uint32_t lookback_queue(const uint64_t* status, uint32_t chunk, uint32_t epoch, int q,
                                                   uint32_t* err)
{
    const int lane = threadIdx.x & 63;
    uint32_t excl = 0;
    long long hi = (long long)chunk - 1;
    uint32_t spins = 0;
    while (hi >= 0) {
        const long long j = hi - lane;
        uint64_t s = pack_status(epoch, kFlagInc, 0);   // before chunk 0: an inclusive zero
        if (j >= 0) s = __hip_atomic_load(status + (size_t)j * 3 + q, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const bool ok = (uint32_t)(s >> 34) == (epoch & kEpochBits) && ((s >> 32) & 3ull) != 0;
        const bool inc = ok && ((s >> 32) & 3ull) == kFlagInc;
        const uint64_t inc_mask = __ballot(inc);
        const uint64_t bad_mask = __ballot(!ok);
        const int first_inc = inc_mask ? __ffsll((unsigned long long)inc_mask) - 1 : 64;
        const uint64_t need = first_inc >= 63 ? ~0ull : ((2ull << first_inc) - 1ull);
        if ((bad_mask & need) && ++spins < kMaxSpins) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        if (bad_mask & need) atomicOr(err, 2u);   // gave up waiting: missing values count as zero
        spins = 0;
        const uint32_t v = (((need >> lane) & 1ull) && ok) ? (uint32_t)s : 0u;
        excl += wave_sum(v);
        if (first_inc < 64) break;
        hi -= 64;
    }
    return excl;
}

// Publish this chunk's aggregates, look back for the exclusive prefix of each
// queue, publish the inclusive prefix.  Called by all threads; wave 0 does the
// work; the result lands in sh.prefix / sh.total.
template <int BLOCK>
__device__ __forceinline__ void lookback3(uint64_t* status, uint32_t chunk, uint32_t epoch, const int tot[3],
                                          ScanShared<BLOCK>& sh, uint32_t* err)
{
    if (threadIdx.x < 64) {
        const int q = threadIdx.x;
        // this lane's queue total, selected without indexing a register array
        const uint32_t mine = (uint32_t)(q == 0 ? tot[0] : (q == 1 ? tot[1] : tot[2]));
        if (q < 3)
            __hip_atomic_store(status + (size_t)chunk * 3 + q,
                               pack_status(epoch, chunk == 0 ? kFlagInc : kFlagAgg, mine), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        uint32_t e0 = 0, e1 = 0, e2 = 0;
        if (chunk > 0) {
            e0 = lookback_queue(status, chunk, epoch, 0, err);
            e1 = lookback_queue(status, chunk, epoch, 1, err);
            e2 = lookback_queue(status, chunk, epoch, 2, err);
        }
        const uint32_t ex = q == 0 ? e0 : (q == 1 ? e1 : e2);
        if (q < 3) {
            if (chunk > 0)
                __hip_atomic_store(status + (size_t)chunk * 3 + q, pack_status(epoch, kFlagInc, ex + mine),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            sh.prefix[q] = (int)ex;
            sh.total[q] = (int)mine;
        }
    }
    __syncthreads();
}

// Arrival-order placement: the block reserves its output range in each queue
// with one atomic add on the queue's counter; the queue ends up holding the
// blocks' outputs in the order the reservations landed, each block's outputs
// in slot order.  No block waits for another.  A reservation that runs past
// `cap` sets bit 0 of *err (stores beyond cap are skipped by the caller).
template <int BLOCK>
__device__ __forceinline__ void reserve3(uint32_t* count_out, uint32_t cap, const int tot[3], ScanShared<BLOCK>& sh,
                                         uint32_t* err)
{
    if (threadIdx.x < 3) {
        const int q = threadIdx.x;
        const uint32_t mine = (uint32_t)(q == 0 ? tot[0] : (q == 1 ? tot[1] : tot[2]));
        uint32_t base = 0;
        if (mine) {
            base = atomicAdd(count_out + q, mine);
            if ((uint64_t)base + mine > cap) atomicOr(err, 1u);
        }
        sh.prefix[q] = (int)base;
        sh.total[q] = (int)mine;
    }
    __syncthreads();
}

}  // namespace gv
