// Onesweep LSD radix sort of (key, u32 value) pairs, 8-bit digits, for u32
// and u64 keys and any run of digits [first_bit, first_bit + bits).
//
// One histogram sweep counts the digits of every pass; each pass is then a
// single read and a single write of the data.  Within a pass, persistent
// workgroups take fixed-size partitions from a ticket counter in launch
// order; a partition ranks its keys stably (wavefront ballots match equal
// digits), publishes its per-digit counts and resolves its global offsets
// by decoupled look-back over the partitions before it, then writes its
// keys digit-grouped from LDS so that every store covers a contiguous run.
// Look-back status words carry an epoch, so no clearing is needed between
// passes or sorts.  The key count is read on the device: a frame needs no
// host round trip.
#include "common.h"
#include "launch.h"

namespace dgs {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kMinSortItems = 4;
constexpr int kMinSortPart = kSortThreads * kMinSortItems;  // smallest partition: 1024 keys
static_assert(kSortThreads == 256, "one thread per digit");
constexpr int kHistBlocks = 128;
constexpr int kSortSpinLimit = 1 << 22;
constexpr int kLookWindow = 4;

int sort_passes(int bits) { return (bits + 7) / 8; }

static size_t max_parts(int64_t cap, int part = kMinSortPart) { return (size_t)((cap + part - 1) / part); }

size_t sort_status_words(int64_t cap) { return max_parts(cap) * 256; }

// Keys per thread: partitions of 4096 keys, or of 1024 for sorts of fewer
// than 2^19 keys, which would otherwise occupy only a few dozen CUs.
static int sort_items(int64_t cap) { return cap >= ((int64_t)1 << 19) ? 16 : 4; }

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
        const uint64_t k = keys[i];
        for (int p = 0; p < passes; p++) atomicAdd(&sh[wave][p][(uint32_t)(k >> (8 * p)) & 255u], 1u);
    }
    __syncthreads();
    for (int p = 0; p < passes; p++) {
        uint32_t s = 0;
        for (int w = 0; w < kSortWaves; w++) s += sh[w][p][tid];
        if (s) atomicAdd(&hist[p * 256 + tid], s);
    }
}

// Number of set bits of `mask` at lanes below this one.
__device__ inline uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// status word: epoch << 34 | flag << 32 | count; flag 1 = partition total,
// 2 = inclusive prefix over this and every earlier partition
__device__ inline uint64_t ld_st64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_st64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of `col` over partitions [0, part) by decoupled look-back
// with up to kLookWindow status words in flight: every partition is resident
// at once, so the walk mostly crosses published totals, and a wide window
// reaches an inclusive prefix in few round trips.  Returns false on a timeout.
__device__ inline bool look_back(const uint64_t* status, size_t stride, int part, uint32_t epoch, uint32_t* excl) {
    uint32_t sum = 0;
    int j = part - 1, spins = 0;
    while (j >= 0) {
        uint64_t s[kLookWindow];
#pragma unroll
        for (int i = 0; i < kLookWindow; i++) s[i] = j - i >= 0 ? ld_st64(status + (size_t)(j - i) * stride) : 0;
        int i = 0;
        bool done = false;
        for (; i < kLookWindow; i++) {
            if (j - i < 0) { done = true; break; }
            if ((uint32_t)(s[i] >> 34) != epoch || ((s[i] >> 32) & 3u) == 0) break;  // not published yet
            sum += (uint32_t)s[i];
            if (((s[i] >> 32) & 3u) == 2u) { done = true; break; }
        }
        if (done) break;
        if (i == 0) {
            if (++spins > kSortSpinLimit) { *excl = sum; return false; }
            __builtin_amdgcn_s_sleep(1);
        }
        j -= i;
    }
    *excl = sum;
    return true;
}

// n_ptr (device) holds the item count, or is null for n = cap.
template <class KeyT, int kSortItems>
__global__ __launch_bounds__(kSortThreads) void k_onesweep(const KeyT* __restrict__ kin,
                                                           const uint32_t* __restrict__ vin,
                                                           KeyT* __restrict__ kout, uint32_t* __restrict__ vout,
                                                           const uint32_t* __restrict__ n_ptr, uint32_t cap,
                                                           int shift, const uint32_t* __restrict__ dcount,
                                                           uint64_t* status, const uint32_t* ep, uint32_t pass_tag,
                                                           uint32_t* ticket, int* err) {
    constexpr int kSortPart = kSortThreads * kSortItems;
    __shared__ KeyT s_key[kSortPart];
    __shared__ uint32_t s_val[kSortPart];
    __shared__ uint32_t s_cnt[kSortWaves][256];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t s_lstart[256];            // start of each digit in the partition-local order
    __shared__ uint32_t s_gbase[256];             // global start of each digit minus its local start
    __shared__ uint32_t s_wsum[kSortWaves];
    __shared__ uint32_t s_part;
    __shared__ uint32_t s_goff[256];  // global start of each digit: exclusive scan of the digit counts
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t epoch = epoch_tag(*ep, pass_tag);
    // the first partition ticket is taken before the digit counts are read,
    // so the two round trips overlap
    if (tid == 0) s_part = atomicAdd(ticket, 1u);
    uint32_t n = n_ptr ? *n_ptr : cap;
    if (n > cap) n = cap;
    const uint32_t nparts = (n + kSortPart - 1) / kSortPart;
    {
        const uint32_t c = dcount[tid];
        uint32_t x = c;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(x, o, 64);
            if (lane >= o) x += u;
        }
        if (lane == 63) s_wsum[wave] = x;
        __syncthreads();
        uint32_t pre = 0;
        for (int w = 0; w < wave; w++) pre += s_wsum[w];
        s_goff[tid] = pre + x - c;
        __syncthreads();  // s_wsum is reused below
    }
    for (;;) {
        for (int d = tid; d < kSortWaves * 256; d += kSortThreads) (&s_cnt[0][0])[d] = 0;
        __syncthreads();
        const uint32_t part = __builtin_amdgcn_readfirstlane(s_part);  // uniform: scalar loop control
        if (part >= nparts) break;
        const uint32_t pbase = part * kSortPart;
        const uint32_t wbase = pbase + wave * (kSortItems * 64);
        KeyT k[kSortItems];
        uint32_t v[kSortItems], rank[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; i++) {
            const uint32_t idx = wbase + i * 64 + lane;
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
        // thread d: partition total of digit d, per-wave offsets, local start
        const int d = tid;
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; w++) {
            const uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = tot;
            tot += c;
        }
        uint32_t x = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(x, o, 64);
            if (lane >= o) x += u;
        }
        if (lane == 63) s_wsum[wave] = x;
        // publish this partition's totals, then look back for the prefix
        uint64_t* my = status + (size_t)part * 256 + d;
        const uint64_t tag = (uint64_t)epoch << 34;
        uint32_t excl = 0;
        if (part == 0) {
            st_st64(my, tag | (2ull << 32) | tot);
        } else {
            st_st64(my, tag | (1ull << 32) | tot);
            if (!look_back(status + d, 256, (int)part, epoch, &excl)) atomicOr(err, (1 << kErrTimeout) | (1 << kErrWaitSort));
            st_st64(my, tag | (2ull << 32) | (excl + tot));
        }
        __syncthreads();
        uint32_t lstart = x - tot;
        for (int w = 0; w < wave; w++) lstart += s_wsum[w];
        s_lstart[d] = lstart;
        s_gbase[d] = s_goff[d] + excl - lstart;
        __syncthreads();
        // partition-local digit-grouped order in LDS
#pragma unroll
        for (int i = 0; i < kSortItems; i++) {
            if (wbase + i * 64 + lane < n) {
                const uint32_t dd = (uint32_t)(k[i] >> shift) & 255u;
                const uint32_t lp = s_lstart[dd] + s_cnt[wave][dd] + rank[i];
                s_key[lp] = k[i];
                s_val[lp] = v[i];
            }
        }
        __syncthreads();
        const uint32_t cnt = n - pbase < (uint32_t)kSortPart ? n - pbase : (uint32_t)kSortPart;
        for (uint32_t i = tid; i < cnt; i += kSortThreads) {
            const KeyT kk = s_key[i];
            const uint32_t pos = s_gbase[(uint32_t)(kk >> shift) & 255u] + i;
            if (pos < n) {  // always true unless a look-back wait timed out
                kout[pos] = kk;
                vout[pos] = s_val[i];
            }
        }
        if (gridDim.x >= nparts) break;  // the other partitions went to other workgroups
        __syncthreads();  // LDS (and s_part) are reused by the next partition
        if (tid == 0) s_part = atomicAdd(ticket, 1u);
    }
}

template <class KeyT, int ITEMS>
static void sort_passes_launch(hipStream_t st, KeyT* k0, uint32_t* v0, KeyT* k1, uint32_t* v1,
                               const uint32_t* n_ptr, uint32_t cap, int first_bit, int passes, const SortScratch& s,
                               const uint32_t* epoch, uint32_t tag0, int* err) {
    const size_t parts = max_parts(cap, kSortThreads * ITEMS);
    const unsigned grid = (unsigned)(parts < 1024 ? parts : 1024);
    KeyT *ki = k0, *ko = k1;
    uint32_t *vi = v0, *vo = v1;
    for (int p = 0; p < passes; p++) {
        hipLaunchKernelGGL((k_onesweep<KeyT, ITEMS>), dim3(grid), dim3(kSortThreads), 0, st, ki, vi, ko, vo, n_ptr,
                           cap, first_bit + 8 * p, s.hist + p * 256, s.status, epoch, tag0 + (uint32_t)p,
                           s.tickets + p, err);
        KeyT* tk = ki; ki = ko; ko = tk;
        uint32_t* tv = vi; vi = vo; vo = tv;
    }
}

template <class KeyT>
static bool radix_sort(hipStream_t st, KeyT* k0, uint32_t* v0, KeyT* k1, uint32_t* v1, const uint32_t* n_ptr,
                       uint32_t cap, int first_bit, int bits, const SortScratch& s, const uint32_t* epoch,
                       uint32_t tag0, int* err) {
    const int passes = sort_passes(bits);
    switch (sort_items(cap)) {
        case 16: sort_passes_launch<KeyT, 16>(st, k0, v0, k1, v1, n_ptr, cap, first_bit, passes, s, epoch, tag0, err); break;
        default: sort_passes_launch<KeyT, 4>(st, k0, v0, k1, v1, n_ptr, cap, first_bit, passes, s, epoch, tag0, err);
    }
    return (passes & 1) != 0;
}

bool launch_radix_sort(hipStream_t st, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                       const uint32_t* n_ptr, uint32_t cap, int bits, const SortScratch& s,
                       const uint32_t* epoch, int* err, bool hist_ready, int first_bit, uint32_t tag0) {
    const int passes = sort_passes(bits);
    if (passes <= 0 || cap == 0) return false;
    if (!hist_ready)
        hipLaunchKernelGGL(k_radix_hist, dim3(kHistBlocks), dim3(kSortThreads), 0, st, k0, n_ptr, cap, passes,
                           s.hist);
    return radix_sort(st, k0, v0, k1, v1, n_ptr, cap, first_bit, bits, s, epoch, tag0, err);
}

bool launch_radix_sort32(hipStream_t st, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n,
                         const SortScratch& s, const uint32_t* epoch, uint32_t tag0, int* err) {
    if (n == 0) return false;
    return radix_sort(st, k0, v0, k1, v1, nullptr, n, 0, 32, s, epoch, tag0, err);
}

// ------------------------------------------------ per-tile depth order

// The second way to the lists' order, for frames with short tile lists: the
// keys are emitted in primitive-id order and sorted stably on their tile bits
// only; then each tile's run is sorted by (depth bits, id) -- the
// (tile, depth) order of Sec. IV-B with ties by id, as the depth sort
// followed by the tile sort gives it.  The (depth bits, id) pairs of a run
// are distinct, so any correct sort yields that order.
//
// Two kernels, one per kind of run.  Runs of up to 256 entries (nearly all
// of them) are sorted by one wavefront in registers, entry lane + 64 m in
// slot m of the lane (1, 2 or 4 slots): a bitonic network whose exchanges
// between entries less than 64 apart are lane shuffles and the others moves
// between a lane's own slots -- no LDS and no barrier.  That kernel also
// lists the tiles with longer runs (a device counter, zeroed by the frame's
// clear).  A fixed grid of workgroups then takes the listed tiles, one
// workgroup per tile at a time: up to kTileSortLds entries by a bitonic
// network whose exchanges stay in the workgroup's four wavefronts except
// for three stages through LDS, and longer ones in chunks of kTileSortLds merged
// in global memory, each element's place being its index in its run plus the
// number of smaller elements in the other run (binary search); the two
// buffers are the free ping-pong buffer of the tile sort and the run's own
// key slots.  Runs are written back in place: key = tile << 32 | depth bits,
// value = id, and the values also into vcopy when set.
constexpr int kTileSortLds = 4096;
constexpr int kTileSortThreads = 256;
constexpr int kTileSortGroups = 512;  // workgroups taking the listed tiles

__device__ __forceinline__ void put_sorted(uint64_t* kr, uint32_t* vr, uint32_t* vcopy, uint64_t tbits, int i, uint64_t v) {
    kr[i] = tbits | (v >> 32);
    vr[i] = (uint32_t)v;
    if (vcopy) vcopy[i] = (uint32_t)v;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// A run of at most 64 M entries sorted by one wavefront, entry lane + 64 m
// in v[m] (the padding holds the largest value).
template <int M>
__device__ __forceinline__ void wave_sort_run(uint64_t* __restrict__ kr, uint32_t* __restrict__ vr, uint32_t* vc,
                                     uint64_t tbits, int L, int lane) {
    uint64_t v[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = lane + 64 * m;
        v[m] = e < L ? (kr[e] << 32) | vr[e] : ~0ull;  // (depth bits, id)
    }
#pragma unroll
    for (int k = 2; k <= 64 * M; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {  // entries m and m ^ (j / 64) of the lane
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const int pm = m ^ (j >> 6);
                    if (pm > m) {
                        const bool up = ((lane + 64 * m) & k) == 0;
                        const uint64_t a = v[m], b = v[pm];
                        const bool sw = (a > b) == up;
                        v[m] = sw ? b : a;
                        v[pm] = sw ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const uint64_t o = shfl_xor_u64(v[m], j);
                    const int e = lane + 64 * m;
                    const bool low = (e & j) == 0, up = (e & k) == 0;
                    v[m] = (low == up) ? (v[m] < o ? v[m] : o) : (v[m] < o ? o : v[m]);
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = lane + 64 * m;
        if (e < L) put_sorted(kr, vr, vc, tbits, e, v[m]);
    }
}

// Runs of 1..256 entries: one wavefront per tile; longer runs are listed.
__global__ __launch_bounds__(64) void k_tile_sort_wave(const uint32_t* __restrict__ ranges,
                                                       uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                       uint32_t* __restrict__ vcopy, uint32_t* __restrict__ long_count,
                                                       uint32_t* __restrict__ long_list) {
    const int lane = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const uint32_t s = ranges[2 * tile];
    const int L = (int)(ranges[2 * tile + 1] - s);
    if (L > 256) {
        if (lane == 0) long_list[atomicAdd(long_count, 1u)] = tile;
        return;
    }
    if (L < 1) return;
    uint64_t* kr = keys + s;
    uint32_t* vr = vals + s;
    uint32_t* vc = vcopy ? vcopy + s : nullptr;
    const uint64_t tbits = (uint64_t)tile << 32;
    if (L <= 64) wave_sort_run<1>(kr, vr, vc, tbits, L, lane);
    else if (L <= 128) wave_sort_run<2>(kr, vr, vc, tbits, L, lane);
    else wave_sort_run<4>(kr, vr, vc, tbits, L, lane);
}

// A run of at most 256 M entries sorted by the workgroup's four wavefronts:
// wavefront w holds entries w 64 M + lane + 64 m in v[m] (the padding holds
// the largest value).  Exchanges between entries less than 64 M apart stay
// in the wavefront (lane shuffles, or moves between a lane's slots); only the
// stages between wavefronts go through LDS (sd, 256 M entries): three of
// them for any M.  With out set the sorted entries [0, L) go there instead
// of back into the run.
template <int M>
__device__ __forceinline__ void group_sort_run(uint64_t* sd, uint64_t* __restrict__ kr, uint32_t* __restrict__ vr,
                                      uint32_t* vc, uint64_t* out, uint64_t tbits, int L, int tid) {
    constexpr int B = 64 * M, P = 4 * B;
    const int w = tid >> 6, lane = tid & 63;
    uint64_t v[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = w * B + lane + 64 * m;
        v[m] = e < L ? (kr[e] << 32) | vr[e] : ~0ull;  // (depth bits, id)
    }
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= B) {  // partner in another wavefront
#pragma unroll
                for (int m = 0; m < M; m++) sd[w * B + lane + 64 * m] = v[m];
                __syncthreads();
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const int e = w * B + lane + 64 * m;
                    const uint64_t o = sd[e ^ j];
                    const bool low = (e & j) == 0, up = (e & k) == 0;
                    v[m] = (low == up) ? (v[m] < o ? v[m] : o) : (v[m] < o ? o : v[m]);
                }
                __syncthreads();
            } else if (j >= 64) {  // slots m and m ^ (j / 64) of the lane
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const int pm = m ^ (j >> 6);
                    if (pm > m) {
                        const bool up = ((w * B + lane + 64 * m) & k) == 0;
                        const uint64_t x = v[m], y = v[pm];
                        const bool sw = (x > y) == up;
                        v[m] = sw ? y : x;
                        v[pm] = sw ? x : y;
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const uint64_t o = shfl_xor_u64(v[m], j);
                    const int e = w * B + lane + 64 * m;
                    const bool low = (e & j) == 0, up = (e & k) == 0;
                    v[m] = (low == up) ? (v[m] < o ? v[m] : o) : (v[m] < o ? o : v[m]);
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = w * B + lane + 64 * m;
        if (e < L) {
            if (out) out[e] = v[m];
            else put_sorted(kr, vr, vc, tbits, e, v[m]);
        }
    }
}

__device__ __forceinline__ void group_sort_any(uint64_t* sd, uint64_t* kr, uint32_t* vr, uint32_t* vc, uint64_t* out,
                                      uint64_t tbits, int L, int tid) {
    if (L <= 512) group_sort_run<2>(sd, kr, vr, vc, out, tbits, L, tid);
    else if (L <= 1024) group_sort_run<4>(sd, kr, vr, vc, out, tbits, L, tid);
    else if (L <= 2048) group_sort_run<8>(sd, kr, vr, vc, out, tbits, L, tid);
    else group_sort_run<16>(sd, kr, vr, vc, out, tbits, L, tid);
}

// Number of entries of the ascending array y[0, n) below v.
__device__ __forceinline__ int count_below(const uint64_t* y, int n, uint64_t v) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if (y[m] < v) lo = m + 1;
        else hi = m;
    }
    return lo;
}

// One run of more than 256 entries, by the whole workgroup (sd: its LDS).
__device__ __forceinline__ void sort_long_run(uint64_t* sd, uint32_t tile, uint32_t s, int L, uint64_t* __restrict__ keys,
                                     uint32_t* __restrict__ vals, uint64_t* __restrict__ spare,
                                     uint32_t* __restrict__ vcopy, int tid) {
    uint64_t* kr = keys + s;
    uint32_t* vr = vals + s;
    uint32_t* vc = vcopy ? vcopy + s : nullptr;
    const uint64_t tbits = (uint64_t)tile << 32;
    // A run of up to kTileSortLds entries is one chunk sorted straight back
    // into place; a longer one is sorted in chunks into the spare buffer,
    // then merged pairwise.  (One call site: the network is inlined once.)
    const bool chunked = L > kTileSortLds;
    uint64_t* a = spare + s;
    for (int c0 = 0; c0 < L; c0 += kTileSortLds) {
        group_sort_any(sd, kr + c0, vr + c0, vc, chunked ? a + c0 : nullptr, tbits, min(kTileSortLds, L - c0), tid);
        __syncthreads();  // sd is reused by the next chunk
    }
    if (!chunked) return;
    __threadfence_block();
    __syncthreads();
    uint64_t* src = a;
    uint64_t* dst = kr;  // the run's own key slots (every key has been read)
    for (int w = kTileSortLds; w < L; w <<= 1) {
        for (int i = tid; i < L; i += kTileSortThreads) {
            const int x0 = (i / (2 * w)) * (2 * w), y0 = x0 + w;
            const uint64_t v = src[i];
            if (i < y0) {  // in the first run of the pair
                const int yn = y0 < L ? min(w, L - y0) : 0;
                dst[i + count_below(src + y0, yn, v)] = v;
            } else {
                dst[x0 + (i - y0) + count_below(src + x0, w, v)] = v;
            }
        }
        __threadfence_block();
        __syncthreads();
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    for (int i = tid; i < L; i += kTileSortThreads) put_sorted(kr, vr, vc, tbits, i, src[i]);
}

// The listed tiles (runs of more than 256 entries), one per workgroup at a
// time.
__global__ __launch_bounds__(kTileSortThreads) void k_tile_sort_group(const uint32_t* __restrict__ ranges,
                                                                      uint64_t* __restrict__ keys,
                                                                      uint32_t* __restrict__ vals,
                                                                      uint64_t* __restrict__ spare,
                                                                      uint32_t* __restrict__ vcopy,
                                                                      const uint32_t* __restrict__ long_count,
                                                                      const uint32_t* __restrict__ long_list) {
    __shared__ uint64_t sd[kTileSortLds];
    const int tid = threadIdx.x;
    const uint32_t n = *long_count;
    for (uint32_t e = blockIdx.x; e < n; e += gridDim.x) {
        const uint32_t tile = long_list[e];
        const uint32_t s = ranges[2 * tile];
        const int L = (int)(ranges[2 * tile + 1] - s);
        sort_long_run(sd, tile, s, L, keys, vals, spare, vcopy, tid);
        __syncthreads();  // sd is reused by the next tile
    }
}

void launch_tile_depth_sort(hipStream_t st, const uint32_t* ranges, int tiles, uint64_t* keys, uint32_t* vals,
                            uint64_t* spare, uint32_t* vcopy, uint32_t* long_count, uint32_t* long_list) {
    if (tiles <= 0) return;
    hipLaunchKernelGGL(k_tile_sort_wave, dim3((unsigned)tiles), dim3(64), 0, st, ranges, keys, vals, vcopy,
                       long_count, long_list);
    const unsigned grid = (unsigned)(tiles < kTileSortGroups ? tiles : kTileSortGroups);
    hipLaunchKernelGGL(k_tile_sort_group, dim3(grid), dim3(kTileSortThreads), 0, st, ranges, keys, vals, spare, vcopy,
                       (const uint32_t*)long_count, (const uint32_t*)long_list);
}

}  // namespace dgs
