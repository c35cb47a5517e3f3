// Single-pass exclusive prefix sum with decoupled look-back, plus the key
// emission and tile-range kernels of cell rasterization (Sec. IV-B): the
// offsets of every primitive's keys come from a scan over all primitives in
// id order, so the emitted sequence (and the ties of the stable sort) are
// deterministic.
#include "common.h"
#include "launch.h"

namespace dgs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanPart = kScanThreads * kScanItems;
constexpr int kSpinLimit = 1 << 22;

// status word: epoch << 34 | flag << 32 | value; flag 1 = partition total,
// 2 = inclusive prefix.  Words from an older epoch read as unpublished.
__device__ inline uint64_t ld_status(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_status(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive scan across the 64 lanes of a wavefront.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Persistent blocks take partitions from a ticket counter in launch order, so
// a partition only ever waits for partitions that are already running.
__global__ __launch_bounds__(kScanThreads) void k_scan_excl(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, int64_t n,
                                                             uint32_t* __restrict__ total, uint64_t* status,
                                                             const uint32_t* ep, uint32_t* ticket, int* err) {
    __shared__ uint32_t s_part, s_wsum[kScanThreads / 64], s_excl;
    const uint32_t epoch = epoch_tag(*ep, 0);
    const int nparts = (int)((n + kScanPart - 1) / kScanPart);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) s_part = atomicAdd(ticket, 1u);
        __syncthreads();
        const int part = (int)s_part;
        if (part >= nparts) break;
        const int64_t base = (int64_t)part * kScanPart + (int64_t)tid * kScanItems;
        uint32_t x[kScanItems], sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            x[i] = (base + i < n) ? in[base + i] : 0u;
            sum += x[i];
        }
        uint32_t incl = wave_incl_scan(sum);
        if (lane == 63) s_wsum[wave] = incl;
        __syncthreads();
        uint32_t wprefix = 0, btotal = 0;
        for (int w = 0; w < kScanThreads / 64; w++) {
            uint32_t s = s_wsum[w];
            if (w < wave) wprefix += s;
            btotal += s;
        }
        if (tid == 0) {
            const uint64_t tag = (uint64_t)epoch << 34;
            uint32_t excl = 0;
            if (part == 0) {
                st_status(&status[0], tag | (2ull << 32) | btotal);
            } else {
                st_status(&status[part], tag | (1ull << 32) | btotal);
                int j = part - 1, spins = 0;
                while (j >= 0) {
                    const uint64_t s = ld_status(&status[j]);
                    const uint32_t flag = (uint32_t)(s >> 32) & 3u;
                    if ((uint32_t)(s >> 34) != epoch || flag == 0) {
                        if (++spins > kSpinLimit) { atomicOr(err, 1 << kErrTimeout); break; }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    excl += (uint32_t)s;
                    if (flag == 2) break;
                    j--;
                }
                st_status(&status[part], tag | (2ull << 32) | (excl + btotal));
            }
            s_excl = excl;
            if (part == nparts - 1) *total = excl + btotal;
        }
        __syncthreads();
        uint32_t run = s_excl + wprefix + incl - sum;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            if (base + i < n) out[base + i] = run;
            run += x[i];
        }
        __syncthreads();  // s_part / s_wsum are reused by the next partition
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t v, size_t n) {
    if (n == 0) return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
}

size_t scan_status_words(int64_t n) { return (size_t)((n + kScanPart - 1) / kScanPart) + 1; }

void launch_exclusive_scan(hipStream_t st, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                           uint64_t* status, const uint32_t* epoch, uint32_t* ticket, int* err) {
    if (n <= 0) {
        launch_fill_u32(st, total, 0u, 1);
        return;
    }
    const size_t nparts = (size_t)((n + kScanPart - 1) / kScanPart);
    const unsigned grid = (unsigned)(nparts < 1024 ? nparts : 1024);
    hipLaunchKernelGGL(k_scan_excl, dim3(grid), dim3(kScanThreads), 0, st, in, out, n, total, status,
                       epoch, ticket, err);
}

__global__ void k_clear(ClearList l) {
    const size_t gid = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    for (int b = 0; b < l.count; b++)
        for (size_t i = gid; i < l.n[b]; i += stride) l.p[b][i] = 0u;
    if (l.bump && gid == 0) *l.bump += 1u;
}

void launch_clear(hipStream_t st, const ClearList& l) {
    size_t most = 0;
    for (int b = 0; b < l.count; b++) most = l.n[b] > most ? l.n[b] : most;
    if (most == 0) most = 1;
    unsigned grid = (unsigned)((most + 255) / 256);
    if (grid > 256) grid = 256;
    hipLaunchKernelGGL(k_clear, dim3(grid), dim3(256), 0, st, l);
}

// ---------------------------------------------------------------- keys

__global__ __launch_bounds__(256) void k_emit_keys(int P, const uint32_t* __restrict__ ntiles,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint64_t* __restrict__ prect,
                                                   const uint32_t* __restrict__ depth, int TX, uint32_t cap,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   int* err) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint32_t nt = ntiles[p];
    if (nt == 0) return;
    uint32_t off = offsets[p];
    if ((uint64_t)off + nt > cap) atomicOr(err, 1 << kErrCapacity);
    uint64_t r = prect[p];
    uint64_t d = depth[p];
    int tx0 = rect_x0(r) / kTile, tx1 = rect_x1(r) / kTile;
    int ty0 = rect_y0(r) / kTile, ty1 = rect_y1(r) / kTile;
    uint32_t i = off;
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++, i++) {
            if (i >= cap) return;
            keys[i] = ((uint64_t)(ty * TX + tx) << 32) | d;
            vals[i] = (uint32_t)p;
        }
}

void launch_emit_keys(hipStream_t st, int P, const uint32_t* ntiles, const uint32_t* offsets,
                      const uint64_t* prect, const uint32_t* depth, int TX, uint32_t cap, uint64_t* keys,
                      uint32_t* vals, int* err) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_emit_keys, dim3((P + 255) / 256), dim3(256), 0, st, P, ntiles, offsets, prect, depth, TX,
                       cap, keys, vals, err);
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_ptr, uint32_t cap,
                                                     uint32_t* __restrict__ ranges) {
    uint32_t n = *n_ptr;
    if (n > cap) n = cap;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        uint32_t t = (uint32_t)(keys[i] >> 32);
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[2 * t] = i;
        if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[2 * t + 1] = i + 1;
    }
}

void launch_tile_ranges(hipStream_t st, const uint64_t* keys, const uint32_t* n_ptr, uint32_t cap,
                        uint32_t* ranges) {
    unsigned grid = (unsigned)((cap + 255) / 256);
    if (grid > 2048) grid = 2048;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_tile_ranges, dim3(grid), dim3(256), 0, st, keys, n_ptr, cap, ranges);
}

}  // namespace dgs
