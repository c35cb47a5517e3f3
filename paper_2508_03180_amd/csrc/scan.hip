// Single-pass exclusive prefix sum with decoupled look-back, plus the key
// emission and tile-range kernels of cell rasterization (Sec. IV-B).  The
// primitives are first sorted by depth (ties by id); the offsets of their
// keys come from a scan over that order, so the emitted sequence is already
// in (depth, id) order within every tile and a stable sort on the tile bits
// alone completes the (tile, depth) order.
#include <string.h>

#include "common.h"
#include "launch.h"

namespace dgs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanPart = kScanThreads * kScanItems;
// Histogram-producing kernels run capped grids (grid-stride), each
// workgroup adding its LDS histogram to the global one once: every global
// bin then takes at most kHistBlocks atomics.  The key emission is bound by
// its stores, so it keeps one primitive per thread up to the cap.
constexpr int kHistBlocks = 512;
constexpr int kPrimKeysPerBlock = 1024;
constexpr int kEmitPrimsPerBlock = 256;

static int hist_grid(int n, int per_block) {
    const int b = (n + per_block - 1) / per_block;
    return b < 1 ? 1 : (b > kHistBlocks ? kHistBlocks : b);
}
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

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Persistent blocks take partitions from a ticket counter in launch order, so
// a partition only ever waits for partitions that are already running.
__global__ __launch_bounds__(kScanThreads) void k_scan_excl(const uint32_t* __restrict__ in,
                                                             uint32_t* __restrict__ out, int64_t n,
                                                             uint32_t* __restrict__ total, uint64_t* status,
                                                             const uint32_t* ep, uint32_t* ticket, int* err,
                                                             const uint32_t* __restrict__ idx) {
    __shared__ uint32_t s_part, s_wsum[kScanThreads / 64], s_excl;
    const uint32_t epoch = epoch_tag(*ep, 0);
    const int nparts = (int)((n + kScanPart - 1) / kScanPart);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) s_part = atomicAdd(ticket, 1u);
        __syncthreads();
        const int part = (int)__builtin_amdgcn_readfirstlane(s_part);  // uniform: scalar loop control
        if (part >= nparts) break;
        const int64_t base = (int64_t)part * kScanPart + (int64_t)tid * kScanItems;
        uint32_t x[kScanItems], sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            uint32_t j = (uint32_t)(base + i);
            if (idx && base + i < n) j = idx[base + i];  // a permutation of [0, n)
            x[i] = (base + i < n && j < (uint64_t)n) ? in[j] : 0u;
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
        if (wave == 0) {
            // decoupled look-back by the whole wavefront: lane l reads the
            // status of partition j - l, so one round trip covers 64
            // predecessors; it stops at the nearest inclusive prefix
            const uint64_t tag = (uint64_t)epoch << 34;
            uint32_t excl = 0;
            if (part == 0) {
                if (lane == 0) st_status(&status[0], tag | (2ull << 32) | btotal);
            } else {
                if (lane == 0) st_status(&status[part], tag | (1ull << 32) | btotal);
                int j = part - 1, spins = 0;
                for (;;) {
                    const int idx = j - lane;
                    uint32_t flag = 2, val = 0;  // before partition 0: an inclusive prefix of 0
                    if (idx >= 0) {
                        const uint64_t st = ld_status(&status[idx]);
                        flag = (uint32_t)(st >> 34) == epoch ? (uint32_t)(st >> 32) & 3u : 0u;
                        val = (uint32_t)st;
                    }
                    const uint64_t notready = __ballot(flag == 0), inclusive = __ballot(flag == 2);
                    const int fn = notready ? __builtin_ctzll(notready) : 64;
                    const int li = inclusive ? __builtin_ctzll(inclusive) : 64;
                    if (li < fn) {  // every partition down to the nearest inclusive prefix is published
                        excl += wave_sum_u32(lane <= li ? val : 0u);
                        break;
                    }
                    if (fn > 0) {  // totals of the published run [0, fn): take them and move on
                        excl += wave_sum_u32(lane < fn ? val : 0u);
                        j -= fn;
                        continue;
                    }
                    if (++spins > kSpinLimit) {
                        if (lane == 0) atomicOr(err, (1 << kErrTimeout) | (1 << kErrWaitScan));
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (lane == 0) st_status(&status[part], tag | (2ull << 32) | (excl + btotal));
            }
            if (lane == 0) {
                s_excl = excl;
                if (part == nparts - 1) *total = excl + btotal;
            }
        }
        __syncthreads();
        uint32_t run = s_excl + wprefix + incl - sum;
#pragma unroll
        for (int i = 0; i < kScanItems; i++) {
            if (base + i < n) out[base + i] = run;
            run += x[i];
        }
        if (gridDim.x >= (unsigned)nparts) break;  // the other partitions went to other workgroups
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
                           uint64_t* status, const uint32_t* epoch, uint32_t* ticket, int* err,
                           const uint32_t* idx) {
    if (n <= 0) {
        launch_fill_u32(st, total, 0u, 1);
        return;
    }
    const size_t nparts = (size_t)((n + kScanPart - 1) / kScanPart);
    const unsigned grid = (unsigned)(nparts < 1024 ? nparts : 1024);
    hipLaunchKernelGGL(k_scan_excl, dim3(grid), dim3(kScanThreads), 0, st, in, out, n, total, status,
                       epoch, ticket, err, idx);
}

__global__ void k_clear(ClearList l, FrameK f, FrameK* fdst) {
    const size_t gid = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    for (int b = 0; b < l.count; b++)
        for (size_t i = gid; i < l.n[b]; i += stride) l.p[b][i] = 0u;
    if (l.bump && gid == 0) *l.bump += 1u;
    if (fdst) {
        static_assert(sizeof(FrameK) % 4 == 0, "frame record in words");
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&f);
        uint32_t* dst = reinterpret_cast<uint32_t*>(fdst);
        for (size_t i = gid; i < sizeof(FrameK) / 4; i += stride) dst[i] = src[i];
    }
}

void launch_clear(hipStream_t st, const ClearList& l, const FrameK* f, FrameK* fdst) {
    size_t most = 0;
    for (int b = 0; b < l.count; b++) most = l.n[b] > most ? l.n[b] : most;
    if (most == 0) most = 1;
    unsigned grid = (unsigned)((most + 255) / 256);
    if (grid > 256) grid = 256;
    FrameK fv;
    if (f) fv = *f;
    else memset(&fv, 0, sizeof(fv));
    hipLaunchKernelGGL(k_clear, dim3(grid), dim3(256), 0, st, l, fv, f ? fdst : nullptr);
}

// ---------------------------------------------------------------- keys

// Depth keys of the primitives with their four byte histograms (per
// workgroup in LDS, added to the global ones once).
__global__ __launch_bounds__(256) void k_prim_keys(int P, const uint32_t* __restrict__ ntiles,
                                                   const uint32_t* __restrict__ depth, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ vals, uint32_t* __restrict__ hist) {
    __shared__ uint32_t sh[4][256];
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&sh[0][0])[i] = 0u;
    __syncthreads();
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const uint32_t k = ntiles[p] ? depth[p] : 0xffffffffu;
        keys[p] = k;
        vals[p] = (uint32_t)p;
#pragma unroll
        for (int b = 0; b < 4; b++) atomicAdd(&sh[b][(k >> (8 * b)) & 255u], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
        const uint32_t c = (&sh[0][0])[i];
        if (c) atomicAdd(&hist[i], c);
    }
}

void launch_prim_keys(hipStream_t st, int P, const uint32_t* ntiles, const uint32_t* depth, uint32_t* keys,
                      uint32_t* vals, uint32_t* hist) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_prim_keys, dim3(hist_grid(P, kPrimKeysPerBlock)), dim3(256), 0, st, P, ntiles, depth, keys, vals, hist);
}

// Key emission in depth order, fused with the digit histograms of the tile
// bytes (hist[b][d]: kept keys whose tile byte b is d).  Along one row of a
// primitive's tile rectangle the tile ids are consecutive: the low tile byte
// then covers a run of bins, counted with a difference array (a +1 / -1 pair
// per run, prefix-summed at the end), and each higher tile byte changes at
// most a few times, counted once per run.  Only keys below the capacity are
// counted (they are the ones sorted).
__global__ __launch_bounds__(256) void k_emit_keys(int P, const uint32_t* __restrict__ order,
                                                   const uint32_t* __restrict__ ntiles,
                                                   const uint32_t* __restrict__ offsets,
                                                   const uint64_t* __restrict__ prect,
                                                   const uint32_t* __restrict__ depth, int TX, uint32_t cap,
                                                   uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                   uint32_t* __restrict__ hist, int passes, int* err) {
    __shared__ uint32_t sh[3][256];  // tile bytes 1, 2 (byte 0 below)
    __shared__ int32_t s_diff[257];  // low tile byte: difference array over the bins
    __shared__ uint32_t s_all;       // low tile byte: runs of 256 or more add to every bin
    __shared__ uint32_t s_wsum[4];
    for (int i = threadIdx.x; i < 3 * 256; i += blockDim.x) (&sh[0][0])[i] = 0u;
    for (int i = threadIdx.x; i < 257; i += blockDim.x) s_diff[i] = 0;
    if (threadIdx.x == 0) s_all = 0u;
    __syncthreads();
    // grid-stride over the depth order: a capped grid, so each workgroup adds
    // its histogram to the global one once
    for (int i0 = blockIdx.x * blockDim.x + threadIdx.x; i0 < P; i0 += gridDim.x * blockDim.x) {
        const uint32_t p = order ? order[i0] : (uint32_t)i0;  // null order: id order
        if (p >= (uint32_t)P) continue;  // a permutation of [0, P) unless a sort wait timed out
        const uint32_t nt = ntiles[p];
        if (nt) {
            const uint32_t off = offsets[i0];
            if ((uint64_t)off + nt > cap) atomicOr(err, 1 << kErrCapacity);
            const uint64_t r = prect[p];
            const uint32_t d = depth[p];
            const int tx0 = rect_x0(r) / kTile, tx1 = rect_x1(r) / kTile;
            const int ty0 = rect_y0(r) / kTile, ty1 = rect_y1(r) / kTile;
            uint32_t i = off;
            for (int ty = ty0; ty <= ty1 && i < cap; ty++) {
                // one row of tiles: consecutive tile ids t0 .. t0 + kept - 1
                const uint32_t t0 = (uint32_t)(ty * TX + tx0);
                const uint32_t len = (uint32_t)(tx1 - tx0 + 1);
                const uint32_t kept = cap - i < len ? cap - i : len;
                for (uint32_t j = 0; j < kept; j++) {
                    keys[i + j] = ((uint64_t)(t0 + j) << 32) | d;
                    vals[i + j] = p;
                }
                if (kept) {
                    if (kept >= 256u) atomicAdd(&s_all, kept >> 8);
                    const uint32_t rem = kept & 255u, a = t0 & 255u;
                    if (rem) {
                        atomicAdd(&s_diff[a], 1);
                        if (a + rem <= 256u) {
                            atomicAdd(&s_diff[a + rem], -1);
                        } else {
                            atomicAdd(&s_diff[256], -1);
                            atomicAdd(&s_diff[0], 1);
                            atomicAdd(&s_diff[a + rem - 256u], -1);
                        }
                    }
                }
                // higher tile bytes change rarely along a row: one count per run
                for (int b = 1; b < passes; b++) {
                    const int sh8 = 8 * b;
                    for (uint32_t t = t0, te = t0 + kept; t < te;) {
                        const uint32_t run_end = ((t >> sh8) + 1u) << sh8;
                        const uint32_t stop = run_end < te ? run_end : te;
                        atomicAdd(&sh[b - 1][(t >> sh8) & 255u], stop - t);
                        t = stop;
                    }
                }
                i += kept;
            }
        }
    }
    __syncthreads();
    {
        // low tile byte: inclusive prefix sum of the difference array
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        int32_t x = s_diff[tid];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t u = __shfl_up(x, o, 64);
            if (lane >= o) x += u;
        }
        if (lane == 63) s_wsum[wave] = (uint32_t)x;
        __syncthreads();
        for (int w = 0; w < wave; w++) x += (int32_t)s_wsum[w];
        const uint32_t c = (uint32_t)x + s_all;
        if (c) atomicAdd(&hist[tid], c);
    }
    for (int b = 1; b < passes; b++)
        for (int i = threadIdx.x; i < 256; i += blockDim.x) {
            const uint32_t c = sh[b - 1][i];
            if (c) atomicAdd(&hist[b * 256 + i], c);
        }
}

void launch_emit_keys(hipStream_t st, int P, const uint32_t* order, const uint32_t* ntiles,
                      const uint32_t* offsets, const uint64_t* prect, const uint32_t* depth, int TX, uint32_t cap,
                      uint64_t* keys, uint32_t* vals, uint32_t* hist, int tile_passes, int* err) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_emit_keys, dim3(hist_grid(P, kEmitPrimsPerBlock)), dim3(256), 0, st, P, order, ntiles, offsets, prect, depth, TX,
                       cap, keys, vals, hist, tile_passes, err);
}

__global__ __launch_bounds__(256) void k_tile_ranges(const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ n_ptr, uint32_t cap,
                                                     uint32_t* __restrict__ ranges,
                                                     const uint32_t* __restrict__ vin, uint32_t* __restrict__ vout,
                                                     uint64_t* load, uint32_t tiles) {
    uint32_t n = *n_ptr;
    if (load && blockIdx.x == 0 && threadIdx.x == 0)  // the frame's load, for the host (pinned memory)
        __hip_atomic_store(load, ((uint64_t)tiles << 32) | n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (n > cap) n = cap;
    // the tile words of the neighbours (at clamped indexes) and the value
    // are loaded at once, before any of them is compared
    const uint32_t* tw = reinterpret_cast<const uint32_t*>(keys) + 1;  // tile of key i: tw[2 i]
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t t = tw[2 * (size_t)i];
        const uint32_t tp = tw[2 * (size_t)(i > 0 ? i - 1 : 0)];
        const uint32_t tn = tw[2 * (size_t)(i + 1 < n ? i + 1 : i)];
        const uint32_t v = vout ? vin[i] : 0u;
        if (i == 0 || tp != t) ranges[2 * t] = i;
        if (i == n - 1 || tn != t) ranges[2 * t + 1] = i + 1;
        if (vout) vout[i] = v;
    }
}

void launch_tile_ranges(hipStream_t st, const uint64_t* keys, const uint32_t* n_ptr, uint32_t cap,
                        uint32_t* ranges, const uint32_t* vin, uint32_t* vout, uint64_t* load, uint32_t tiles) {
    unsigned grid = (unsigned)((cap + 255) / 256);
    if (grid > 2048) grid = 2048;
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL(k_tile_ranges, dim3(grid), dim3(256), 0, st, keys, n_ptr, cap, ranges, vin, vout, load, tiles);
}

}  // namespace dgs
