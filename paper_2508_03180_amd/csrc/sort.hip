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
#include "order.h"

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
// One launch of independent workgroups of 16 wavefronts.  Wavefront w of
// workgroup b takes one tile (the tiles spread over the image, so that the
// few long runs spread over the workgroups).  A run of up to 256 entries is
// sorted by its wavefront alone, entry lane + 64 m in register slot m of
// the lane (1, 2 or 4 slots): a bitonic network whose exchanges between
// entries less than 64 apart are cross-lane moves (DPP and row swaps, no
// LDS) and the others moves between a lane's own slots.  The workgroup then
// sorts its longer runs with the same network spread over several
// wavefronts, only the exchanges between wavefronts going through LDS: runs
// of up to 512 entries two at a time, one on each half of the workgroup,
// longer ones with all 16 wavefronts, up to 2048 entries (2 per lane: more
// would spill registers at the 64 VGPRs that let two workgroups share a
// CU).  Runs longer than that are sorted in chunks of 2048 into the free
// ping-pong buffer of the tile sort and merged pairwise between that buffer
// and the run's own key slots, each element's place being its index in its
// half plus the number of smaller elements in the other half (binary
// search).  Runs are written back in place: key = tile << 32 | depth bits,
// value = id, the values also into vcopy when set.  One more workgroup of
// the launch builds the compositor's work queue from the tile ranges
// (build_work_queue, order.h) meanwhile.  Every helper is inlined: the
// kernel makes no calls.
constexpr int kTsWaves = 16;
constexpr int kTsThreads = 64 * kTsWaves;
constexpr int kTsShort = 256;              // longest run one wavefront sorts
constexpr int kTsChunk = 2 * kTsThreads;  // longest run the workgroup sorts in registers
constexpr int kTsHalf = kTsThreads / 2;   // longest run half of the workgroup sorts

__device__ __forceinline__ void put_sorted(uint64_t* kr, uint32_t* vr, uint32_t* vcopy, uint64_t tbits, int i, uint64_t v) {
    kr[i] = tbits | (v >> 32);
    vr[i] = (uint32_t)v;
    if (vcopy) vcopy[i] = (uint32_t)v;
}

// The value that lane ^ J holds, for J a power of two below 64, without
// LDS: DPP moves for partners inside a row of 16 lanes, gfx950's row swaps
// for 16 and 32 (each returns the two operands after swapping the odd rows
// of the first with the even rows of the second, resp. the upper half of
// the first with the lower half of the second).
template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane) {
    if constexpr (J == 1) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (J == 2) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (J == 4) {
        const int m = __builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror: lane ^ 7
        return (uint32_t)__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);     // quad_perm [3,2,1,0]: ^ 3
    } else if constexpr (J == 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else if constexpr (J == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    } else {
        static_assert(J == 32, "lane distance");
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
}

template <int J>
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v, int lane) {
    const uint32_t lo = lane_xor<J>((uint32_t)v, lane), hi = lane_xor<J>((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// j is a constant once the networks' loops are unrolled
__device__ __forceinline__ uint64_t lane_xor64(uint64_t v, int j, int lane) {
    switch (j) {
        case 1: return lane_xor64<1>(v, lane);
        case 2: return lane_xor64<2>(v, lane);
        case 4: return lane_xor64<4>(v, lane);
        case 8: return lane_xor64<8>(v, lane);
        case 16: return lane_xor64<16>(v, lane);
        default: return lane_xor64<32>(v, lane);
    }
}

// One bitonic compare-exchange of entry e (value v) with entry e ^ j, whose
// value is o: the lower entry of the pair keeps the smaller value in an
// ascending block, the larger in a descending one.  ej: bit j of e is set
// (the upper entry); ek: bit k of e is set (a descending block of the k-merge).
__device__ __forceinline__ uint64_t cx(uint64_t v, uint64_t o, bool ej, bool ek) {
    return ((v < o) == (ej == ek)) ? v : o;
}

// Bits 0..5 of the lane index (each a lane mask the compiler can keep in
// scalar registers).
struct LaneBits {
    bool b[6];
    __device__ __forceinline__ explicit LaneBits(int lane) {
#pragma unroll
        for (int i = 0; i < 6; i++) b[i] = (lane >> i) & 1;
    }
    __device__ __forceinline__ bool operator[](int pow2) const { return b[__builtin_ctz(pow2)]; }
};

// The stages of a bitonic network over P entries held by consecutive
// wavefronts, entry base + lane + 64 m in v[m] of wavefront base / (64 M)
// (base a multiple of 64 M), that stay inside the wavefront: exchanges
// 64 or more apart between a lane's slots, shorter ones across lanes.
// Stages j >= 64 M need another wavefront's entries: xchg(k, j) does those.
template <int M, class Xchg>
__device__ __forceinline__ void bitonic(uint64_t (&v)[M], int P, int base, int lane, Xchg xchg) {
    const LaneBits lb(lane);
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64 * M) {
                xchg(k, j);
            } else if (j >= 64) {  // slots m and m ^ (j / 64) of the lane
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const int pm = m ^ (j >> 6);
                    if (pm > m) {
                        const bool up = ((base + 64 * m) & k) == 0;
                        const uint64_t x = v[m], y = v[pm];
                        const bool sw = (x > y) == up;
                        v[m] = sw ? y : x;
                        v[pm] = sw ? x : y;
                    }
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const bool ek = k < 64 ? lb[k] : ((base + 64 * m) & k) != 0;
                    v[m] = cx(v[m], lane_xor64(v[m], j, lane), lb[j], ek);
                }
            }
        }
    }
}

// A run of at most P <= 64 M entries sorted by one wavefront (the padding
// holds the largest value); with M = 1 and P < 64 the network stops at
// blocks of P lanes.
template <int M, int P = 64 * M>
__device__ __forceinline__ void wave_sort_run(uint64_t* __restrict__ kr, uint32_t* __restrict__ vr, uint32_t* vc,
                                              uint64_t tbits, int L, int lane) {
    uint64_t v[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = lane + 64 * m;
        v[m] = e < L ? (kr[e] << 32) | vr[e] : ~0ull;  // (depth bits, id)
    }
    bitonic<M>(v, P, 0, lane, [](int, int) {});
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = lane + 64 * m;
        if (e < L) put_sorted(kr, vr, vc, tbits, e, v[m]);
    }
}

// A run of at most 64 W M entries sorted by W wavefronts of the workgroup
// (tid: the thread's index among them): wavefront w holds entries
// w 64 M + lane + 64 m (the padding holds the largest value); the stages
// between wavefronts go through LDS (sd, 64 W M entries).  With out set the
// sorted entries [0, L) go there instead of back into the run.
// Its barriers are the workgroup's: every wavefront of the workgroup runs
// the same network at the same time.
template <int M, int W = kTsWaves>
__device__ __forceinline__ void group_sort_run(uint64_t* sd, uint64_t* __restrict__ kr, uint32_t* __restrict__ vr,
                                               uint32_t* vc, uint64_t* out, uint64_t tbits, int L, int tid) {
    constexpr int B = 64 * M;
    const int w = tid >> 6, lane = tid & 63, base = w * B;
    uint64_t v[M];
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = base + lane + 64 * m;
        v[m] = e < L ? (kr[e] << 32) | vr[e] : ~0ull;  // (depth bits, id)
    }
    bitonic<M>(v, 64 * W * M, base, lane, [&](int k, int j) {
#pragma unroll
        for (int m = 0; m < M; m++) sd[base + lane + 64 * m] = v[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; m++) {
            const int e = base + lane + 64 * m;
            v[m] = cx(v[m], sd[e ^ j], (e & j) != 0, (e & k) != 0);
        }
        __syncthreads();
    });
#pragma unroll
    for (int m = 0; m < M; m++) {
        const int e = base + lane + 64 * m;
        if (e < L) {
            if (out) out[e] = v[m];
            else put_sorted(kr, vr, vc, tbits, e, v[m]);
        }
    }
}

__device__ __forceinline__ void group_sort_any(uint64_t* sd, uint64_t* kr, uint32_t* vr, uint32_t* vc, uint64_t* out,
                                               uint64_t tbits, int L, int tid) {
    if (L <= kTsThreads) group_sort_run<1>(sd, kr, vr, vc, out, tbits, L, tid);
    else group_sort_run<2>(sd, kr, vr, vc, out, tbits, L, tid);
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

// One run of more than kTsHalf entries, by the whole workgroup (sd: its LDS).
__device__ __forceinline__ void sort_long_run(uint64_t* sd, uint32_t tile, uint32_t s, int L,
                                              uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                              uint64_t* __restrict__ spare, uint32_t* __restrict__ vcopy, int tid) {
    uint64_t* kr = keys + s;
    uint32_t* vr = vals + s;
    uint32_t* vc = vcopy ? vcopy + s : nullptr;
    const uint64_t tbits = (uint64_t)tile << 32;
    // A run of up to kTsChunk entries is one chunk sorted straight back into
    // place; a longer one is sorted in chunks into the spare buffer, then
    // merged pairwise.  (One call site: the network is inlined once.)
    const bool chunked = L > kTsChunk;
    uint64_t* a = spare + s;
    for (int c0 = 0; c0 < L; c0 += kTsChunk) {
        group_sort_any(sd, kr + c0, vr + c0, vc, chunked ? a + c0 : nullptr, tbits, min(kTsChunk, L - c0), tid);
        __syncthreads();  // sd is reused by the next chunk
    }
    if (!chunked) return;
    __threadfence_block();
    __syncthreads();
    uint64_t* src = a;
    uint64_t* dst = kr;  // the run's own key slots (every key has been read)
    for (int w = kTsChunk; w < L; w <<= 1) {
        for (int i = tid; i < L; i += kTsThreads) {
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
    for (int i = tid; i < L; i += kTsThreads) put_sorted(kr, vr, vc, tbits, i, src[i]);
}

// The workgroup's long runs as lanes 0..15 of every wavefront hold them.
struct LongRuns {
    int tile, s, len;
};

// The runs of mask (lanes of q) sorted kTsWaves / W at a time, one per group
// of W wavefronts, each by a network of 64 W entries; a group left without
// a run in the last round runs the network on padding only.
template <int W>
__device__ __forceinline__ void sort_in_groups(uint64_t mask, const LongRuns& q, uint64_t* sd,
                                               uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                               uint32_t* __restrict__ vcopy, int tid) {
    constexpr int NG = kTsWaves / W;
    const int g = (tid >> 6) / W;
    while (mask) {
        const int first = __builtin_ctzll(mask);
        int mine = -1;
#pragma unroll
        for (int r = 0; r < NG; r++) {
            if (mask) {
                const int i = __builtin_ctzll(mask);
                mask &= mask - 1;
                if (r == g) mine = i;
            }
        }
        const int ic = mine < 0 ? first : mine;
        const uint32_t rt = (uint32_t)__shfl(q.tile, ic, 64), rs = (uint32_t)__shfl(q.s, ic, 64);
        const int rl = mine < 0 ? 0 : __shfl(q.len, ic, 64);
        group_sort_run<1, W>(sd + g * 64 * W, keys + rs, vals + rs, vcopy ? vcopy + rs : nullptr, nullptr,
                             (uint64_t)rt << 32, rl, tid - g * 64 * W);
        __syncthreads();  // sd is reused by the next round
    }
}

// A workgroup's LDS: the work queue's counts and partial sums (order.h), or
// the sort's exchange buffer.
constexpr int kQueueBytes = (kOrderClasses + 1024) * 4;
constexpr int kTsSharedBytes = kQueueBytes > kTsChunk * 8 ? kQueueBytes : kTsChunk * 8;

// two workgroups per CU: 64 VGPRs at most.  The last workgroup builds the
// compositor's work queue (it needs the tile ranges only) while the others
// sort the runs.
__global__ __launch_bounds__(kTsThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_tile_sort(
    const uint32_t* __restrict__ ranges, int tiles, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
    uint64_t* __restrict__ spare, uint32_t* __restrict__ vcopy, uint32_t split_len, uint32_t* __restrict__ order,
    uint32_t* __restrict__ queue, uint64_t* long_stat, uint32_t prims) {
    __shared__ __align__(16) unsigned char smem[kTsSharedBytes];
    __shared__ int lt_tile[kTsWaves], lt_s[kTsWaves], lt_len[kTsWaves];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int G = (int)gridDim.x - 1;  // workgroups sorting runs
    if ((int)blockIdx.x == G) {
        uint32_t* s_cnt = reinterpret_cast<uint32_t*>(smem);
        build_work_queue(ranges, tiles, split_len, order, queue, s_cnt, s_cnt + kOrderClasses, tid, long_stat, prims);
        return;
    }
    uint64_t* sd = reinterpret_cast<uint64_t*>(smem);
    // wavefront w takes a tile of the w-th band of G tiles, at an offset
    // that moves by a fixed stride from band to band
    const int t = w * G + (int)(((int64_t)blockIdx.x + (int64_t)w * (G * 5 / 8 + 1)) % G);
    uint32_t s = 0;
    int L = 0;
    if (t < tiles) {
        s = ranges[2 * t];
        L = (int)(ranges[2 * t + 1] - s);
    }
    if (L > kTsShort) {  // sorted below, by the workgroup
        if (lane == 0) {
            lt_tile[w] = t;
            lt_s[w] = (int)s;
            lt_len[w] = L;
        }
    } else {
        if (lane == 0) lt_tile[w] = -1;
        const uint64_t tbits = (uint64_t)(uint32_t)t << 32;
        uint64_t* kr = keys + s;
        uint32_t* vr = vals + s;
        uint32_t* vc = vcopy ? vcopy + s : nullptr;
        if (L == 1) {  // in place; only its value copy is due
            if (vc && lane == 0) vc[0] = vr[0];
        } else if (L > 1) {
            if (L <= 16) wave_sort_run<1, 16>(kr, vr, vc, tbits, L, lane);
            else if (L <= 32) wave_sort_run<1, 32>(kr, vr, vc, tbits, L, lane);
            else if (L <= 64) wave_sort_run<1>(kr, vr, vc, tbits, L, lane);
            else if (L <= 128) wave_sort_run<2>(kr, vr, vc, tbits, L, lane);
            else wave_sort_run<4>(kr, vr, vc, tbits, L, lane);
        }
    }
    __syncthreads();
    // the long runs, from the lists in LDS read once into lanes 0..15:
    // runs longer than kTsHalf one at a time with the whole workgroup, the
    // others two at a time on the two halves of the workgroup (a network of
    // kTsHalf entries each)
    const int li = lane & (kTsWaves - 1);
    const LongRuns q{lt_tile[li], lt_s[li], lt_len[li]};
    const uint64_t has = __ballot(lane < kTsWaves && q.tile >= 0);
    const uint64_t whole0 = has & ~__ballot(q.len <= kTsHalf);
    uint64_t whole = whole0;
    while (whole) {
        const int i = __builtin_ctzll(whole);
        whole &= whole - 1;
        sort_long_run(sd, (uint32_t)__shfl(q.tile, i, 64), (uint32_t)__shfl(q.s, i, 64), __shfl(q.len, i, 64), keys,
                      vals, spare, vcopy, tid);
        __syncthreads();  // sd is reused by the next run
    }
    sort_in_groups<kTsWaves / 2>(has & ~whole0, q, sd, keys, vals, vcopy, tid);
}

void launch_tile_depth_sort(hipStream_t st, const uint32_t* ranges, int tiles, uint64_t* keys, uint32_t* vals,
                            uint64_t* spare, uint32_t* vcopy, uint32_t split_len, uint32_t* order, uint32_t* queue,
                            uint64_t* long_stat, uint32_t prims) {
    if (tiles <= 0) return;
    const unsigned grid = (unsigned)((tiles + kTsWaves - 1) / kTsWaves) + 1;  // + the work queue's
    hipLaunchKernelGGL(k_tile_sort, dim3(grid), dim3(kTsThreads), 0, st, ranges, tiles, keys, vals, spare, vcopy,
                       split_len, order, queue, long_stat, prims);
}

}  // namespace dgs
