// The compositor's work queue (Sec. V-B's tiles taken by persistent
// wavefronts, heaviest first), built by one workgroup of 1024 threads: by
// k_tile_order, or by the per-tile depth sort's last workgroup.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace dgs {

// Builds the work queue: per tile one whole-tile item, or for lists of at
// least split_len entries two half-tile items.  Items are counting-sorted by
// estimated cost -- list length times the vector instructions a list
// entry's member costs over the item's strips -- and laid out costliest
// first, so the longest walks start at once (order within a cost class is
// arbitrary: it only affects scheduling, never results).
// queue[0] = head (reset), queue[1] = item count.  One workgroup.  With
// long_stat set (pinned host memory), also stores prims << 32 | the number
// of keys in runs of more than kLongRunKeys entries, for the host's choice
// of list order.
constexpr int kOrderClasses = 4096;
constexpr uint32_t kLongRunKeys = 4096;

__device__ __forceinline__ void tile_items(uint32_t len, uint32_t split_len, uint32_t& n, uint32_t& cls) {
    // vector instructions per member of a whole-tile (4 strips) and a half
    // (2 strips) walk, counted in the compiled member loop
    const uint32_t w = len >= split_len ? 45u : 77u;
    n = len >= split_len ? 2u : 1u;
    const uint32_t c = (len * w) >> 5;
    cls = c < (uint32_t)kOrderClasses ? c : (uint32_t)kOrderClasses - 1u;
}

// s_cnt [kOrderClasses]: counts, then the first slot of each class;
// s_part [1024]: the threads' partial sums (LDS of the calling workgroup).
__device__ __forceinline__ void build_work_queue(const uint32_t* __restrict__ ranges, int ntiles, uint32_t split_len,
                                        uint32_t* __restrict__ order, uint32_t* __restrict__ queue,
                                        uint32_t* s_cnt, uint32_t* s_part, int tid,
                                        uint64_t* long_stat = nullptr, uint32_t prims = 0) {
    __shared__ uint32_t s_long;
    for (int i = tid; i < kOrderClasses; i += 1024) s_cnt[i] = 0;
    if (tid == 0) s_long = 0;
    __syncthreads();
    uint32_t lng = 0;  // keys of this thread's tiles in runs longer than kLongRunKeys
    for (int t = tid; t < ntiles; t += 1024) {
        uint32_t n, cls;
        const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
        tile_items(len, split_len, n, cls);
        atomicAdd(&s_cnt[cls], n);
        lng += len > kLongRunKeys ? len : 0u;
    }
    if (long_stat && lng) atomicAdd(&s_long, lng);
    __syncthreads();
    if (long_stat && tid == 0)
        __hip_atomic_store(long_stat, ((uint64_t)prims << 32) | s_long, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    // costliest first: thread i owns classes 4095 - 4i .. 4092 - 4i
    constexpr int kPer = kOrderClasses / 1024;
    uint32_t loc[kPer], run = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
        loc[j] = run;
        run += s_cnt[kOrderClasses - 1 - (kPer * tid + j)];
    }
    s_part[tid] = run;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan of the per-thread totals
        const uint32_t x = tid >= o ? s_part[tid - o] : 0u;
        __syncthreads();
        s_part[tid] += x;
        __syncthreads();
    }
    const uint32_t before = s_part[tid] - run;
#pragma unroll
    for (int j = 0; j < kPer; j++) s_cnt[kOrderClasses - 1 - (kPer * tid + j)] = before + loc[j];
    if (tid == 1023) {
        queue[0] = 0;
        queue[1] = s_part[1023];
    }
    __syncthreads();
    for (int t = tid; t < ntiles; t += 1024) {
        uint32_t n, cls;
        tile_items(ranges[2 * t + 1] - ranges[2 * t], split_len, n, cls);
        const uint32_t o = atomicAdd(&s_cnt[cls], n);
        // mode 0: whole tile; 2 + h: half h
        if (n == 1u) order[o] = (uint32_t)t << 3;
        else for (uint32_t h = 0; h < 2u; h++) order[o + h] = ((uint32_t)t << 3) | (2u + h);
    }
}

}  // namespace dgs
