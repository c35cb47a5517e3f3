// Tile compositors.
//
// Duplex (Sec. V-A, eq. hybrid_renderer with w_n = v_n T_n, eq. dulpex_T;
// Sec. V-B early termination; Sec. VI-A false-positive skip).  For every
// pixel the cells of its tile are walked front to back.  Inside a cell the
// members are summed without order:
//     A = sum alpha c,  B = sum alpha,  P = prod (1 - v alpha)
// over members whose box contains the pixel and whose alpha reaches
// alpha_min, with alpha = min(alpha_max, sigma G'(x')).  Across cells
//     N += v T A,  D += v T B,  T *= P,
// a cell is blended only while T (the transmittance in front of it) is at
// least eps, and the colour is C = N / D (bg where D = 0).
//
// Alpha (eqs. alpha_blending, transmittance): the same walk over
// depth-sorted Gaussians with C += T alpha c, T *= 1 - alpha, plus T bg.
//
// Mapping: a wavefront runs without workgroup barriers and owns either a
// whole 16x16 tile or, for tiles with long lists, one 16x8 half of it
// (strips 2h and 2h + 1, strip j = rows 4j..4j+3; lane l holds pixel
// (l & 15, 4j + (l >> 4)) of every strip it owns).  Work items are taken
// from a queue that lists them heaviest first.  The tile list is consumed in
// chunks of up to 64 Gaussian records (whole cells): each lane loads one
// record, the wave ballots which strips every record's box touches, and the
// records go to the wave's private LDS slot, from which they are read as
// broadcasts.  The next chunk is fetched into registers while the current
// one is composited.  Cells and members that touch none of the tile's
// strips are skipped with scalar bit tests on the ballots.
#include "cells.h"
#include "order.h"
#include "common.h"
#include "launch.h"

namespace dgs {

constexpr int kWaves = 4;  // tiles per workgroup


struct Chunk {
    float4 r0, r1, r2;  // this lane's record
    float v;            // v of this lane's cell (Duplex walks)
    bool ok;
    int nch;            // entries in the chunk (cells, or Gaussians in the alpha walk)
    int first, cnt;     // cell walks, lane c < nch: first record lane and member count of cell c
};

// The next chunk of a cell walk: whole cells from list position pos (at
// most 64 records, at most end - pos cells).
template <bool RAGGED>
__device__ inline void load_cell_chunk(const CompositeArgs& a, uint32_t pos, uint32_t end, int lane, Chunk& q) {
    // every field is set on every path: a partly set struct would be kept in
    // scratch memory instead of registers
    CellChunk ch;
    load_cells<RAGGED>(a.vals, a.offs, a.cell_v, a.K, pos, end, -1, lane, ch);
    q.nch = ch.nch;
    q.first = ch.first;
    q.cnt = ch.cnt;
    q.ok = ch.g >= 0;
    q.v = ch.v;
    q.r0 = q.r1 = q.r2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (!q.ok) return;
    const float4* p = reinterpret_cast<const float4*>(a.recs + ch.g);
    q.r0 = p[0];
    q.r1 = p[1];
    q.r2 = p[2];
}

// The next chunk of the per-Gaussian walk: up to 64 list entries from pos.
__device__ inline void load_gauss_chunk(const CompositeArgs& a, uint32_t pos, uint32_t end, int lane, Chunk& q) {
    const int n = (int)min(64u, end - pos);
    q.nch = n;
    q.first = q.cnt = 0;
    q.ok = lane < n;
    q.r0 = q.r1 = q.r2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    q.v = 0.0f;
    if (!q.ok) return;
    const float4* p = reinterpret_cast<const float4*>(a.recs + a.vals[pos + lane]);
    q.r0 = p[0];
    q.r1 = p[1];
    q.r2 = p[2];
}

// Ballots of the owned strips each lane's record touches: B[j] for strip
// s0 + j (rows 4(s0 + j)..4(s0 + j) + 3 of the tile), j < NS; s0 = 0 for a
// whole tile (NS = 4), 2h for half h (NS = 2).  s0 is wavefront-uniform, so
// the ballots stay in scalar registers.
// Also returns, per lane, its record's strip bits (sm) and the tile columns
// its box covers (cols, bit x for column tx0 + x; 0 when it misses the tile).
template <int NS>
__device__ inline void strip_ballots(const Chunk& q, int tx0, int ty0, int s0, uint64_t* B, uint32_t& sm,
                                     uint32_t& cols) {
    sm = 0;
    cols = 0;
    if (q.ok) {
        const int x0 = __float_as_int(q.r2.y), y0 = __float_as_int(q.r2.z);
        const uint32_t wxy = __float_as_uint(q.r2.w);
        const int x1 = x0 + (int)(wxy & 0xffffu), y1 = y0 + (int)(wxy >> 16);
        if (x0 <= tx0 + 15 && x1 >= tx0) {
            const int lo = max(x0, tx0) - tx0, hi = min(x1, tx0 + 15) - tx0;
            cols = ((2u << (hi - lo)) - 1u) << lo;
#pragma unroll
            for (int j = 0; j < NS; j++) {
                const int r0 = ty0 + 4 * (s0 + j);
                if (y0 <= r0 + 3 && y1 >= r0) sm |= 1u << j;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NS; j++) B[j] = __ballot((sm >> j) & 1u);
}

// Columns (bit x: tile column x) holding an active pixel in a strip, from
// the ballot of the strip's active lanes (lane l: column l & 15).
__device__ inline uint32_t active_columns(uint64_t m) {
    m |= m >> 32;
    m |= m >> 16;
    return (uint32_t)m & 0xffffu;
}

__device__ inline void store_chunk(GRec* lds, int lane, const Chunk& q) {
    if (!q.ok) return;
    float4* d = reinterpret_cast<float4*>(lds + lane);
    d[0] = q.r0;
    d[1] = q.r1;
    d[2] = q.r2;
}

struct RecView {
    float ox, oy, ca, cb, cc, lo, r, g, b;
    int x0, y0;
    uint32_t wx, wy;
};

typedef float F4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const F4 LdsF4;

// The wavefront's record array as a 32-bit LDS address, held in a scalar
// register: every lane reads the same record, so its address is uniform.
__device__ inline uint32_t lds_base(const GRec* lds) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(const LdsF4*)lds);
}

__device__ inline RecView read_rec(uint32_t lb, int i) {
    const LdsF4* p = (const LdsF4*)(uintptr_t)(lb + (uint32_t)i * (uint32_t)sizeof(GRec));
    const F4 a = p[0], b = p[1], c = p[2];
    RecView e;
    e.ox = a.x; e.oy = a.y; e.ca = a.z; e.cb = a.w;
    e.cc = b.x; e.lo = b.y; e.r = b.z; e.g = b.w;
    e.b = c.x;
    e.x0 = __float_as_int(c.y);
    e.y0 = __float_as_int(c.z);
    const uint32_t wxy = __float_as_uint(c.w);
    e.wx = wxy & 0xffffu;
    e.wy = wxy >> 16;
    return e;
}


// The frame's values the compositors use, loaded once per wavefront from the
// device frame record (scalar registers; the kernel argument is left as is).
// The output pointers are global-memory pointers: stored through generic
// pointers, they became flat stores, which the compiler counts as possible
// LDS accesses too, so every later wait for an LDS read had to wait for all
// of them.
typedef __attribute__((address_space(1))) float GFloat;
typedef __attribute__((address_space(1))) int32_t GInt;
struct FrameView {
    int TX, W, H;
    float eps, th, amax, bg0, bg1, bg2;
    GFloat* color;
    GFloat* D;
    GFloat* T;
    GInt* last;
    GFloat* sv_color;  // saved state of the frame for its backward (SAVE walks only)
    GFloat* sv_D;
    GFloat* sv_T;
    GInt* sv_last;
};

__device__ inline FrameView frame_view(const FrameK* fr) {
    FrameView f;
    f.TX = fr->k.TX;
    f.W = fr->k.W;
    f.H = fr->k.H;
    f.eps = fr->o.no_et ? 0.0f : fr->o.eps;
    f.th = fr->o.log2_alpha_min;
    f.amax = fr->o.alpha_max;
    f.bg0 = fr->o.bg[0];
    f.bg1 = fr->o.bg[1];
    f.bg2 = fr->o.bg[2];
    f.color = (GFloat*)fr->color;
    f.D = (GFloat*)fr->D;
    f.T = (GFloat*)fr->T;
    f.last = (GInt*)fr->last;
    f.sv_color = (GFloat*)fr->sv_color;
    f.sv_D = (GFloat*)fr->sv_D;
    f.sv_T = (GFloat*)fr->sv_T;
    f.sv_last = (GInt*)fr->sv_last;
    return f;
}

// Work item: tile << 3 | mode; mode 0 = the whole tile (all four strips),
// mode 2 + h = half h (strips 2h and 2h + 1).

// Statistics counters (STATS only): n_val, n_rendered (the termination ratio
// 1 - n_rendered / n_val), in-box member evaluations and (pixel, entry) pairs
// that contributed, for the algorithmic work count.
struct Counters {
    uint32_t val = 0, rend = 0, box = 0, cellhit = 0, cellpx = 0;
};

// The hybrid renderer over one tile (NS = 4) or one half (NS = 2, strips s0
// and s0 + 1)
// (Sec. V-A, eq. hybrid_renderer with w_n = v_n T_n and eq. dulpex_T; Sec. V-B
// termination; Sec. VI-A box gate): cells front to back; a pixel whose
// transmittance in front of a cell is below eps stops there; inside a cell
// every member that passes the box and alpha_min gates adds w alpha c to N
// and w alpha to D with the cell's weight w = v T (the cell's alpha sums A,
// B of the equation times w, accumulated member by member), and
// P = prod (1 - v alpha) updates T after the cell; C = N / D at the end.
// LC: the "w/o T^cell" weights -- cell_v holds w_n = v_n max(0, 1 - d_n / tau),
// no transmittance and no termination.
// A cell counts as contributing at a pixel (`last`) when any of its members
// passed both gates there, whatever its weight.
// SAVE: also write the state the backward replays from -- colour, D, and the
// list position of the last contributing cell whose transmittance in front
// is at least kMinReplayT together with that transmittance.
// RAGGED: cells with their own member counts (CSR offsets), else K per cell.
template <bool STATS, int NS, bool LC, bool SAVE, bool RAGGED>
__device__ inline void duplex_tile(const CompositeArgs& a, const FrameView& f, int tile, int s0, int lane, GRec* lds,
                                 Counters& cn) {
    const int tx0 = (tile % f.TX) * kTile, ty0 = (tile / f.TX) * kTile;
    const int px = tx0 + (lane & 15), py0 = ty0 + 4 * s0 + (lane >> 4);
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const int K = a.K;
    const uint32_t kmask = member_mask(K);
    const float eps = f.eps, th = f.th, amax = f.amax;
    const uint32_t lb = lds_base(lds);

    float T[NS], N0[NS], N1[NS], N2[NS], D[NS];
    float thj[NS];  // gate threshold of strip j's pixel for the current cell, +inf once it has terminated
    int32_t last[NS];
    int32_t rlast[NS];  // SAVE: replay start (list position + 1, 0 = none)
    float rT[NS];       // SAVE: transmittance in front of that entry
    bool inb[NS];  // the pixel lies in the image
#pragma unroll
    for (int j = 0; j < NS; j++) {
        T[j] = 1.0f; N0[j] = N1[j] = N2[j] = D[j] = 0.0f; last[j] = 0;
        rlast[j] = 0; rT[j] = 1.0f;
        inb[j] = px < f.W && py0 + 4 * j < f.H;
        thj[j] = inb[j] ? th : INFINITY;
    }
    // the per-cell ballots below are ballots of single compares, combined
    // with these as scalar masks (a ballot of a combination of lane masks
    // is rebuilt through a vector register first)
    uint64_t inbm[NS];  // strip j's pixels in the image
#pragma unroll
    for (int j = 0; j < NS; j++) inbm[j] = __ballot(inb[j]);

    Chunk q;
    if (start < end) load_cell_chunk<RAGGED>(a, start, end, lane, q);
    bool alive = true;
    for (uint32_t pos = start; pos < end && (alive || STATS);) {
        const int nch = q.nch;
        int cfirst = 0, ccnt = 0;  // of this chunk (q takes the next one below)
        if constexpr (RAGGED) {
            cfirst = q.first;
            ccnt = q.cnt;
        }
        // Duplex: log2 v goes into the record's log2 sigma, so that the
        // walk computes v alpha directly (the alpha_min test moves by log2 v)
        // per record lane, its cell's gate threshold and weight clamp (read
        // by the cell loop from the cell's first lane)
        float cthc = th, cvmax = amax;
        if (!LC) {
            const float lv = fold_log2_weight(q.v);
            q.r1.y += lv;
            cthc = th + lv;
            cvmax = q.v * amax;
        }
        store_chunk(lds, lane, q);
        uint64_t B[NS];
        uint32_t rsm, rcols;  // this lane's record: strips and tile columns its box touches
        strip_ballots<NS>(q, tx0, ty0, s0, B, rsm, rcols);
        const float cv = q.v;
        const uint32_t next = pos + nch;
        if (next < end) load_cell_chunk<RAGGED>(a, next, end, lane, q);
        for (int c = 0; c < nch; c++) {
            if (STATS) {  // (pixel, cell) pairs the walk reaches: listed, in the image, not terminated
#pragma unroll
                for (int j = 0; j < NS; j++) cn.cellpx += LC ? inb[j] : inb[j] && !(T[j] < eps);
            }
            // fixed K: cell c holds record lanes cK .. cK + K - 1
            const int base = RAGGED ? lane_value(cfirst, c) : c * K;
            const uint32_t cm = RAGGED ? member_mask(lane_value(ccnt, c)) : kmask;
            uint32_t mj[NS], any = 0;
#pragma unroll
            for (int j = 0; j < NS; j++) {
                mj[j] = (uint32_t)(B[j] >> base) & cm;
                any |= mj[j];
            }
            if (!any) continue;  // no member of this cell touches the owned strips
            const float v = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cv), base));
            // Duplex: every record of this cell holds log2 sigma + log2 v, so
            // its power pw is log2(v sigma G'); alpha >= alpha_min becomes
            // pw >= th + log2 v and min(alpha_max, .) becomes min(v alpha_max, .)
            const float thc = LC ? th : __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cthc), base));
            const float vmax = LC ? amax : __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cvmax), base));
            // a pixel still blends while T >= eps (T never rises, so once
            // below eps it stays below: no state is carried across cells)
            bool act[NS];
#pragma unroll
            for (int j = 0; j < NS; j++) act[j] = LC ? inb[j] : inb[j] && !(T[j] < eps);
            if constexpr (!LC) {
                uint64_t am[NS], amall = 0;  // ballots of act
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    thj[j] = act[j] ? thc : INFINITY;
                    am[j] = __ballot(!(T[j] < eps)) & inbm[j];
                    amall |= am[j];
                }
                if (!STATS && !amall) {
                    alive = false;
                    break;
                }
                // once pixels have terminated, a member whose box misses every
                // pixel still blending cannot change anything: drop it (a
                // finished pixel has threshold +inf, so it is never hit)
                if (!STATS) {
                    uint32_t live = 0;
#pragma unroll
                    for (int j = 0; j < NS; j++) {
                        if (am[j] == inbm[j]) {  // every pixel of strip j still blends
                            live |= mj[j];
                            continue;
                        }
                        // B[j]: the records touching strip j
                        const uint32_t ac = active_columns(am[j]);
                        mj[j] = (uint32_t)((__ballot((rcols & ac) != 0u) & B[j]) >> base) & cm;
                        live |= mj[j];
                    }
                    any = live;
                    if (!any) continue;  // no member reaches a blending pixel: T, last unchanged
                }
            }
            // the cell's weight is fixed before its members: w alpha c and
            // w alpha go straight into N and D (no per-cell sums A, B); in the
            // Duplex walk al below is v alpha and w alpha = T (v alpha)
            float wj[NS], P[NS];
            // some member of this cell passed both gates at the pixel (0 / 1 in
            // a vector register: a lane-mask bool carried through the member
            // loop is merged with the exec mask by scalar instructions every
            // iteration)
            uint32_t hc[NS];
#pragma unroll
            for (int j = 0; j < NS; j++) { wj[j] = LC ? v : T[j]; P[j] = 1.0f; hc[j] = 0u; }
            for (uint32_t rem = any; rem; rem &= rem - 1) {
                const int k = __builtin_ctz(rem);
                const RecView e = read_rec(lb, base + k);
                const uint32_t rx = (uint32_t)(px - e.x0);
                const bool inx = rx <= e.wx;
                const float dx = (float)(int)rx + e.ox;
                // outside the box's columns the power is -inf: the alpha_min
                // test then rejects the pixel as the box test would
                const float t0 = inx ? fmaf(e.ca * dx, dx, e.lo) : -INFINITY;
                const float t1 = e.cb * dx;
                const uint32_t ry0 = (uint32_t)(py0 - e.y0);
                const float dy0 = (float)(int)ry0 + e.oy;
                // every strip is evaluated (strips the member misses fail the
                // row test in every lane): no scalar test per strip
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    const uint32_t ry = ry0 + 4u * j;
                    const float dy = j ? dy0 + 4.0f * j : dy0;  // the row 4j below, without a conversion
                    const float pw = fmaf(dy, fmaf(e.cc, dy, t1), t0);
                    const bool iny = ry <= e.wy;
                    const bool hit = iny & (pw >= thj[j]);  // false once the pixel has terminated
                    if (STATS) {
                        const bool val = iny & (pw >= thc);
                        cn.val += val;
                        cn.rend += val && act[j];
                        cn.box += inx && iny && act[j];
                    }
                    // no branch: a pixel that is not hit adds alpha = 0, which
                    // leaves N, D and P exactly unchanged (the owned strips then
                    // interleave without exec-mask changes)
                    // min(vmax, 2^pw) as a clamp to [0, vmax] (2^pw >= 0)
                    const float al = hit ? __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(pw), 0.0f, vmax) : 0.0f;
                    const float wa = wj[j] * al;
                    N0[j] = fmaf(wa, e.r, N0[j]);
                    N1[j] = fmaf(wa, e.g, N1[j]);
                    N2[j] = fmaf(wa, e.b, N2[j]);
                    D[j] += wa;
                    if constexpr (!LC) P[j] = fmaf(-P[j], al, P[j]);
                    hc[j] = hit ? 1u : hc[j];
                }
            }
            // no branch: a pixel that no longer blends had threshold +inf in
            // this cell, so P = 1 and no hit there (T and last unchanged)
#pragma unroll
            for (int j = 0; j < NS; j++) {
                if (!mj[j]) continue;  // scalar: nothing of this cell in strip j
                const int32_t idx = (int32_t)(pos + c - start + 1);
                if constexpr (SAVE) {
                    const bool rep = hc[j] != 0u && T[j] >= kMinReplayT;
                    rlast[j] = rep ? idx : rlast[j];
                    rT[j] = rep ? T[j] : rT[j];
                }
                if constexpr (!LC) T[j] *= P[j];
                last[j] = hc[j] != 0u ? idx : last[j];
                if (STATS) cn.cellhit += hc[j] != 0u;
            }
        }
        pos = next;
    }
    const size_t HW = (size_t)f.W * f.H;
#pragma unroll
    for (int j = 0; j < NS; j++) {
        const int py = py0 + 4 * j;
        if (px >= f.W || py >= f.H) continue;
        const size_t p = (size_t)py * f.W + px;
        if (D[j] > 0.0f) {
            const float inv = 1.0f / D[j];
            f.color[p] = N0[j] * inv;
            f.color[HW + p] = N1[j] * inv;
            f.color[2 * HW + p] = N2[j] * inv;
        } else {
            f.color[p] = f.bg0;
            f.color[HW + p] = f.bg1;
            f.color[2 * HW + p] = f.bg2;
        }
        if (f.D) f.D[p] = D[j];
        if (f.T) f.T[p] = T[j];
        if (f.last) f.last[p] = last[j];
        if constexpr (SAVE) {
            f.sv_color[p] = f.color[p];
            f.sv_color[HW + p] = f.color[HW + p];
            f.sv_color[2 * HW + p] = f.color[2 * HW + p];
            f.sv_D[p] = D[j];
            f.sv_T[p] = rT[j];
            f.sv_last[p] = rlast[j];
        }
    }
}

template <bool STATS, int NS>
__device__ inline void alpha_tile(const CompositeArgs& a, const FrameView& f, int tile, int s0, int lane, GRec* lds,
                                 Counters& cn) {
    const int tx0 = (tile % f.TX) * kTile, ty0 = (tile / f.TX) * kTile;
    const int px = tx0 + (lane & 15), py0 = ty0 + 4 * s0 + (lane >> 4);
    const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
    const float eps = f.eps, th = f.th, amax = f.amax;

    float T[NS], C0[NS], C1[NS], C2[NS];
    int32_t last[NS];
    bool inb[NS];  // the pixel lies in the image
#pragma unroll
    for (int j = 0; j < NS; j++) {
        T[j] = 1.0f; C0[j] = C1[j] = C2[j] = 0.0f; last[j] = 0;
        inb[j] = px < f.W && py0 + 4 * j < f.H;
    }
    uint64_t inbm[NS];  // strip j's pixels in the image (ballots of single compares below)
#pragma unroll
    for (int j = 0; j < NS; j++) inbm[j] = __ballot(inb[j]);
    const uint32_t lb = lds_base(lds);
    Chunk q;
    if (start < end) load_gauss_chunk(a, start, end, lane, q);
    bool alive = true;
    for (uint32_t pos = start; pos < end && (alive || STATS);) {
        const int n = q.nch;
        store_chunk(lds, lane, q);
        uint64_t B[NS], any = 0;
        uint32_t rsm, rcols;
        strip_ballots<NS>(q, tx0, ty0, s0, B, rsm, rcols);
#pragma unroll
        for (int j = 0; j < NS; j++) any |= B[j];
        const uint32_t next = pos + n;
        if (next < end) load_gauss_chunk(a, next, end, lane, q);
        int since_check = 0;
        for (; any; any &= any - 1) {
            int m = __builtin_ctzll(any);
            // every 8 Gaussians: stop when no pixel of the owned strips still
            // blends, else keep only the records whose box meets a column
            // that still holds a blending pixel in a strip the box covers
            // (a record outside every such column and strip cannot hit a
            // blending pixel, so dropping it changes no output)
            if (!STATS && ++since_check == 8) {
                since_check = 0;
                uint64_t amall = 0, live = 0;
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    // every ballot runs on every lane; B[j]: the records
                    // touching strip j
                    const uint64_t am = __ballot(!(T[j] < eps)) & inbm[j];
                    amall |= am;
                    const uint32_t ac = active_columns(am);
                    live |= __ballot((rcols & ac) != 0u) & B[j];
                }
                if (!amall) {
                    alive = false;
                    break;
                }
                any &= live;
                if (!any) break;
                m = __builtin_ctzll(any);
            }
            const RecView e = read_rec(lb, m);
            const uint32_t rx = (uint32_t)(px - e.x0);
            const bool inx = rx <= e.wx;
            const float dx = (float)(int)rx + e.ox;
            const float t0 = inx ? fmaf(e.ca * dx, dx, e.lo) : -INFINITY;  // as in the Duplex walk
            const float t1 = e.cb * dx;
            const uint32_t ry0 = (uint32_t)(py0 - e.y0);
            const float dy0 = (float)(int)ry0 + e.oy;
#pragma unroll
            for (int j = 0; j < NS; j++) {
                // termination before each Gaussian (T only changes on a hit
                // and never rises, so no state is carried across Gaussians)
                const bool act = inb[j] && !(T[j] < eps);
                const uint32_t ry = ry0 + 4u * j;
                const float dy = j ? dy0 + 4.0f * j : dy0;
                const float pw = fmaf(dy, fmaf(e.cc, dy, t1), t0);
                const bool iny = ry <= e.wy;
                const bool hit = iny & (pw >= th);
                if (STATS) {
                    cn.val += hit;
                    cn.box += inx && iny && act;
                }
                if (hit & act) {
                    const float al = fminf(amax, __builtin_amdgcn_exp2f(pw));
                    const float w = al * T[j];
                    C0[j] = fmaf(w, e.r, C0[j]);
                    C1[j] = fmaf(w, e.g, C1[j]);
                    C2[j] = fmaf(w, e.b, C2[j]);
                    T[j] -= w;
                    last[j] = (int32_t)(pos + m - start + 1);
                    if (STATS) {
                        cn.rend++;
                        cn.cellhit++;
                    }
                }
            }
        }
        pos = next;
    }
    const size_t HW = (size_t)f.W * f.H;
#pragma unroll
    for (int j = 0; j < NS; j++) {
        const int py = py0 + 4 * j;
        if (px >= f.W || py >= f.H) continue;
        const size_t p = (size_t)py * f.W + px;
        f.color[p] = fmaf(T[j], f.bg0, C0[j]);
        f.color[HW + p] = fmaf(T[j], f.bg1, C1[j]);
        f.color[2 * HW + p] = fmaf(T[j], f.bg2, C2[j]);
        if (f.D) f.D[p] = 1.0f - T[j];
        if (f.T) f.T[p] = T[j];
        if (f.last) f.last[p] = last[j];
    }
}

// Persistent wavefronts: each takes the next work item of a queue that lists
// them heaviest first, so long tiles start early and short ones fill in
// behind them on every XCD.  Every wavefront leaves once the queue is empty.
// MODE: kModeDuplex, kModeAlpha or kModeLcwsr.
template <int MODE, bool STATS, bool SAVE, bool RAGGED>
__global__ __launch_bounds__(256) void k_composite(CompositeArgs a) {
    __shared__ GRec s_rec[kWaves][64];
    const FrameView f = frame_view(a.fr);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    GRec* lds = s_rec[wave];
    const uint32_t nitems = a.queue[1];
    Counters cn;
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(a.queue, 1u);
        // lane 0's ticket in a scalar register: the item, its tile and its
        // half are then wavefront-uniform, and so is all loop control below
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= nitems) break;
        const uint32_t item = a.order[t];
        const int tile = (int)(item >> 3), mode = (int)(item & 7u);
        // half-tile items (the tiles with the longest lists, which set the
        // kernel's span) issue ahead of whole-tile items on their SIMD
        if (mode != 0)
            __builtin_amdgcn_s_setprio(3);
        else
            __builtin_amdgcn_s_setprio(0);
        if (MODE == kModeAlpha) {
            if (mode == 0)
                alpha_tile<STATS, 4>(a, f, tile, 0, lane, lds, cn);
            else
                alpha_tile<STATS, 2>(a, f, tile, 2 * (mode - 2), lane, lds, cn);
        } else {
            constexpr bool LC = MODE == kModeLcwsr;
            if (mode == 0)
                duplex_tile<STATS, 4, LC, SAVE, RAGGED>(a, f, tile, 0, lane, lds, cn);
            else
                duplex_tile<STATS, 2, LC, SAVE, RAGGED>(a, f, tile, 2 * (mode - 2), lane, lds, cn);
        }
    }
    if (STATS) {
        atomicAdd(&a.counters[0], (unsigned long long)cn.val);
        atomicAdd(&a.counters[1], (unsigned long long)cn.rend);
        atomicAdd(&a.counters[2], (unsigned long long)cn.box);
        atomicAdd(&a.counters[3], (unsigned long long)cn.cellhit);
        atomicAdd(&a.counters[4], (unsigned long long)cn.cellpx);
    }
}

// Builds the work queue (build_work_queue, order.h) in one workgroup.
__global__ __launch_bounds__(1024) void k_tile_order(const uint32_t* __restrict__ ranges, int ntiles,
                                                     uint32_t split_len, uint32_t* __restrict__ order,
                                                     uint32_t* __restrict__ queue, uint64_t* long_stat,
                                                     uint32_t prims) {
    __shared__ uint32_t s_cnt[kOrderClasses];
    __shared__ uint32_t s_part[1024];
    build_work_queue(ranges, ntiles, split_len, order, queue, s_cnt, s_part, (int)threadIdx.x, long_stat, prims);
}

static unsigned persistent_grid(int tiles) {
    // enough wavefronts to fill every SIMD of the 256 CUs a few times over
    const int waves = 4 * tiles < 256 * 4 * 4 ? 4 * tiles : 256 * 4 * 4;
    return (unsigned)((waves + kWaves - 1) / kWaves);
}

void launch_tile_order(hipStream_t st, const uint32_t* ranges, int tiles, uint32_t split_len, uint32_t* order,
                       uint32_t* queue, uint64_t* long_stat, uint32_t prims) {
    if (tiles <= 0) return;
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), 0, st, ranges, tiles, split_len, order, queue, long_stat,
                       prims);
}

template <int MODE, bool SAVE, bool RAGGED>
static void launch_variant(hipStream_t st, dim3 g, dim3 b, const CompositeArgs& a) {
    if (a.counters)
        hipLaunchKernelGGL((k_composite<MODE, true, SAVE, RAGGED>), g, b, 0, st, a);
    else
        hipLaunchKernelGGL((k_composite<MODE, false, SAVE, RAGGED>), g, b, 0, st, a);
}

template <int MODE>
static void launch_mode(hipStream_t st, const CompositeArgs& a) {
    const int tiles = a.k.TX * a.k.TY;  // host copy of the frame's tile grid
    if (tiles <= 0) return;
    const dim3 g(persistent_grid(tiles)), b(256);
    if constexpr (MODE == kModeAlpha) {
        launch_variant<MODE, false, false>(st, g, b, a);
    } else if constexpr (MODE == kModeDuplex) {
        if (a.save && a.offs) launch_variant<MODE, true, true>(st, g, b, a);
        else if (a.save) launch_variant<MODE, true, false>(st, g, b, a);
        else if (a.offs) launch_variant<MODE, false, true>(st, g, b, a);
        else launch_variant<MODE, false, false>(st, g, b, a);
    } else {
        if (a.offs) launch_variant<MODE, false, true>(st, g, b, a);
        else launch_variant<MODE, false, false>(st, g, b, a);
    }
}

void launch_composite_duplex(hipStream_t st, const CompositeArgs& a) { launch_mode<kModeDuplex>(st, a); }
void launch_composite_alpha(hipStream_t st, const CompositeArgs& a) { launch_mode<kModeAlpha>(st, a); }
void launch_composite_lcwsr(hipStream_t st, const CompositeArgs& a) { launch_mode<kModeLcwsr>(st, a); }

}  // namespace dgs
