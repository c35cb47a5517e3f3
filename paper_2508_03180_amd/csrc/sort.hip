// Onesweep LSD radix sort of (u64 key, u32 value) pairs, 8-bit digits.
//
// One histogram sweep counts the digits of every pass; each pass is then a
// single read and a single scatter of the data.  Within a pass, persistent
// workgroups take fixed-size partitions from a ticket counter; each
// partition ranks its keys stably in LDS (wavefront ballots match equal
// digits), publishes its per-digit counts and resolves its global offsets by
// decoupled look-back over the partitions before it.  The key count is read
// on the device, so a frame needs no host round trip.
#include "common.h"
#include "launch.h"

namespace dgs {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 12;
constexpr int kSortPart = kSortThreads * kSortItems;
constexpr uint32_t kSFlagAgg = 1u << 30, kSFlagInc = 2u << 30, kSValMask = (1u << 30) - 1;
constexpr int kSortSpinLimit = 1 << 22;

int sort_passes(int bits) { return (bits + 7) / 8; }

static size_t max_parts(int64_t cap) { return (size_t)((cap + kSortPart - 1) / kSortPart); }

size_t sort_status_words(int64_t cap, int passes) { return max_parts(cap) * 256 * (size_t)passes; }

__global__ __launch_bounds__(256) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ n_ptr, uint32_t cap, int passes,
                                                    uint32_t* __restrict__ hist) {
    __shared__ uint32_t sh[kSortWaves][8][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    for (int i = tid; i < kSortWaves * 8 * 256; i += kSortThreads) (&sh[0][0][0])[i] = 0;
    __syncthreads();
    uint32_t n = *n_ptr;
    if (n > cap) n = cap;
    for (uint32_t i = blockIdx.x * kSortThreads + tid; i < n; i += gridDim.x * kSortThreads) {
        uint64_t k = keys[i];
        for (int p = 0; p < passes; p++) atomicAdd(&sh[wave][p][(uint32_t)(k >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int p = 0; p < passes; p++) {
        uint32_t s = 0;
        for (int w = 0; w < kSortWaves; w++) s += sh[w][p][tid];
        if (s) atomicAdd(&hist[p * 256 + tid], s);
    }
}

// In place: per pass, counts -> exclusive digit offsets.
__global__ __launch_bounds__(256) void k_radix_hist_scan(uint32_t* hist, int passes) {
    __shared__ uint32_t s_w[kSortWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int p = 0; p < passes; p++) {
        uint32_t v = hist[p * 256 + tid], x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            uint32_t u = __shfl_up(x, d, 64);
            if (lane >= d) x += u;
        }
        if (lane == 63) s_w[wave] = x;
        __syncthreads();
        uint32_t pre = 0;
        for (int w = 0; w < wave; w++) pre += s_w[w];
        hist[p * 256 + tid] = pre + x - v;
        __syncthreads();
    }
}

__device__ inline uint32_t lds_status(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void sts_status(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Number of set bits of `mask` at lanes below this one.
__device__ inline uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__global__ __launch_bounds__(kSortThreads) void k_onesweep(const uint64_t* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           const uint32_t* __restrict__ n_ptr, uint32_t cap,
                                                           int shift, const uint32_t* __restrict__ goff,
                                                           uint32_t* status, uint32_t* ticket, int* err) {
    __shared__ uint32_t s_part;
    __shared__ uint32_t s_cnt[kSortWaves][256];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t s_base[256];              // global start of each digit for this partition
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t n = *n_ptr;
    if (n > cap) n = cap;
    const uint32_t nparts = (n + kSortPart - 1) / kSortPart;
    for (;;) {
        if (tid == 0) s_part = atomicAdd(ticket, 1u);
        for (int d = tid; d < kSortWaves * 256; d += kSortThreads) (&s_cnt[0][0])[d] = 0;
        __syncthreads();
        const uint32_t part = s_part;
        if (part >= nparts) break;
        const uint32_t wbase = part * kSortPart + wave * (kSortItems * 64);
        uint64_t k[kSortItems];
        uint32_t v[kSortItems], rank[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; i++) {
            uint32_t idx = wbase + i * 64 + lane;
            if (idx < n) {
                k[i] = kin[idx];
                v[i] = vin[idx];
            }
        }
        // stable ranking inside the wave: item i of every lane precedes item i+1
#pragma unroll
        for (int i = 0; i < kSortItems; i++) {
            const bool valid = wbase + i * 64 + lane < n;
            const uint32_t d = (uint32_t)(k[i] >> shift) & 255u;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; b++) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            uint32_t before = 0;
            if (valid) before = s_cnt[wave][d];
            rank[i] = before + lanes_below(peers);
            if (valid && lane == __builtin_ctzll(peers)) s_cnt[wave][d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // thread d: partition total of digit d, per-wave exclusive offsets
        {
            const int d = tid;
            uint32_t tot = 0;
#pragma unroll
            for (int w = 0; w < kSortWaves; w++) {
                uint32_t c = s_cnt[w][d];
                s_cnt[w][d] = tot;
                tot += c;
            }
            uint32_t* my = status + (size_t)part * 256 + d;
            uint32_t excl = 0;
            if (part == 0) {
                sts_status(my, kSFlagInc | tot);
            } else {
                sts_status(my, kSFlagAgg | tot);
                int j = (int)part - 1, spins = 0;
                while (j >= 0) {
                    uint32_t s = lds_status(status + (size_t)j * 256 + d);
                    if ((s & ~kSValMask) == 0) {
                        if (++spins > kSortSpinLimit) { atomicOr(err, 1 << kErrTimeout); break; }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    excl += s & kSValMask;
                    if (s & kSFlagInc) break;
                    j--;
                }
                sts_status(my, kSFlagInc | ((excl + tot) & kSValMask));
            }
            s_base[d] = goff[d] + excl;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; i++) {
            if (wbase + i * 64 + lane < n) {
                const uint32_t d = (uint32_t)(k[i] >> shift) & 255u;
                const uint32_t pos = s_base[d] + s_cnt[wave][d] + rank[i];
                kout[pos] = k[i];
                vout[pos] = v[i];
            }
        }
        __syncthreads();  // LDS is reused by the next partition
    }
}

__global__ void k_clear_sort(uint32_t* status, size_t words, const uint32_t* n_ptr, uint32_t cap, int passes,
                             size_t pass_stride, uint32_t* hist, uint32_t* tickets) {
    uint32_t n = *n_ptr;
    if (n > cap) n = cap;
    const size_t used = (size_t)((n + kSortPart - 1) / kSortPart) * 256;
    const size_t gid = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    for (int p = 0; p < passes; p++)
        for (size_t i = gid; i < used; i += stride) status[p * pass_stride + i] = 0;
    for (size_t i = gid; i < (size_t)passes * 256; i += stride) hist[i] = 0;
    if (gid < 8) tickets[gid] = 0;
}

bool launch_radix_sort(hipStream_t st, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                       const uint32_t* n_ptr, uint32_t cap, int bits, const SortScratch& s, int* err) {
    const int passes = sort_passes(bits);
    if (passes <= 0 || cap == 0) return false;
    const size_t pass_stride = max_parts(cap) * 256;
    hipLaunchKernelGGL(k_clear_sort, dim3(512), dim3(256), 0, st, s.status, pass_stride * passes, n_ptr, cap,
                       passes, pass_stride, s.hist, s.tickets);
    unsigned hgrid = (unsigned)((cap + kSortThreads * 16 - 1) / (kSortThreads * 16));
    if (hgrid > 1024) hgrid = 1024;
    hipLaunchKernelGGL(k_radix_hist, dim3(hgrid), dim3(kSortThreads), 0, st, k0, n_ptr, cap, passes, s.hist);
    hipLaunchKernelGGL(k_radix_hist_scan, dim3(1), dim3(256), 0, st, s.hist, passes);
    size_t parts = max_parts(cap);
    unsigned grid = (unsigned)(parts < 2048 ? parts : 2048);
    uint64_t *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL(k_onesweep, dim3(grid), dim3(kSortThreads), 0, st, ki, vi, ko, vo, n_ptr, cap, 8 * p,
                           s.hist + p * 256, s.status + p * pass_stride, s.tickets + p, err);
        uint64_t* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
    return (passes & 1) != 0;
}

}  // namespace dgs
