// Chunks of whole cells for the tile walks (forward and backward).
//
// A cell emits its own Gaussians (Sec. IV-A): either K each, member k of
// cell n being Gaussian n K + k, or a variable number given by CSR offsets,
// the members of cell n being Gaussians offs[n] .. offs[n+1] - 1 (at most
// kMaxK, checked by the cell preprocess, which culls a cell whose range is
// malformed).  A walk stages the records of consecutive list entries in the
// 64 lanes of a wavefront, whole cells at a time: lane c < nch describes
// cell c of the chunk (its first record lane, member count, id, first
// Gaussian and v), and every record lane r knows its Gaussian and its cell's
// v.
#pragma once
#include "common.h"

namespace dgs {

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ inline int wave_incl_sum(int x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ inline int lane_value(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

struct CellChunk {
    int nch;      // cells in the chunk (wavefront-uniform)
    int first;    // lane c < nch: first record lane of cell c
    int cnt;      // lane c < nch: its member count
    uint32_t id;  // lane c < nch: its cell id
    int gfirst;   // lane c < nch: its first Gaussian
    float vc;     // lane c < nch: its v
    int g;        // record lane: its Gaussian, -1 when the lane holds no record
    float v;      // record lane: v of its cell (0 without a record)
};

// Number of list entries, counted back from position hi (exclusive) and not
// below lo, whose members fill at most 64 record lanes (at least one entry
// when hi > lo: a cell has at most kMaxK <= 64 members).
template <bool RAGGED>
__device__ inline int cells_fitting_back(const uint32_t* __restrict__ vals, const int32_t* __restrict__ offs, int K,
                                         uint32_t lo, uint32_t hi, int lane) {
    const uint32_t avail = min(64u, hi - lo);
    if constexpr (!RAGGED) return (int)min((uint32_t)(64 / K), avail);
    int cnt = 0;
    if ((uint32_t)lane < avail) {
        const uint32_t cell = vals[hi - 1 - lane];
        cnt = offs[cell + 1] - offs[cell];
    }
    const int incl = wave_incl_sum(cnt, lane);
    return __popcll(__ballot((uint32_t)lane < avail && incl <= 64));
}

// The chunk starting at list position p: nch_in entries (from
// cells_fitting_back), or with nch_in < 0 as many whole cells as fit in 64
// records, at most end - p.  RAGGED: the CSR layout (offs), else K per cell.
template <bool RAGGED>
__device__ inline void load_cells(const uint32_t* __restrict__ vals, const int32_t* __restrict__ offs,
                                  const float* __restrict__ cell_v, int K, uint32_t p, uint32_t end, int nch_in,
                                  int lane, CellChunk& ch) {
    if constexpr (!RAGGED) {
        ch.nch = nch_in >= 0 ? nch_in : (int)min((uint32_t)(64 / K), end - p);
        ch.first = lane * K;
        ch.cnt = K;
        ch.id = 0;
        ch.gfirst = 0;
        ch.vc = 0.0f;
        ch.g = -1;
        ch.v = 0.0f;
        if (lane < ch.nch) {  // cell lanes
            ch.id = vals[p + lane];
            ch.gfirst = (int)(ch.id * (uint32_t)K);
            ch.vc = cell_v[ch.id];
        }
        if (lane < ch.nch * K) {  // record lanes: member k of cell c
            const int c = lane / K, k = lane - c * K;
            const uint32_t cell = vals[p + c];
            ch.g = (int)(cell * (uint32_t)K) + k;
            ch.v = cell_v[cell];
        }
        return;
    }
    const uint32_t avail = nch_in >= 0 ? (uint32_t)nch_in : min(64u, end - p);
    ch.id = 0;
    ch.gfirst = 0;
    ch.cnt = 0;
    ch.vc = 0.0f;
    if ((uint32_t)lane < avail) {
        ch.id = vals[p + lane];
        ch.gfirst = offs[ch.id];
        ch.cnt = offs[ch.id + 1] - ch.gfirst;
        ch.vc = cell_v[ch.id];
    }
    const int incl = wave_incl_sum(ch.cnt, lane);
    ch.first = incl - ch.cnt;
    ch.nch = nch_in >= 0 ? nch_in : __popcll(__ballot((uint32_t)lane < avail && incl <= 64));
    ch.g = -1;
    ch.v = 0.0f;
    for (int c = 0; c < ch.nch; c++) {  // uniform: a few cells per chunk
        const int f = lane_value(ch.first, c), n = lane_value(ch.cnt, c), gb = lane_value(ch.gfirst, c);
        const float vc = __int_as_float(lane_value(__float_as_int(ch.vc), c));
        const bool mine = lane >= f && lane < f + n;
        ch.g = mine ? gb + (lane - f) : ch.g;
        ch.v = mine ? vc : ch.v;
    }
}

// Member mask of a cell with n members (n <= 32).
__device__ inline uint32_t member_mask(int n) { return n >= 32 ? 0xffffffffu : ((1u << n) - 1u); }

}  // namespace dgs
