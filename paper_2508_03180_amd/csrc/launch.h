// Host-side launchers of the HIP kernels (internal to the library).
#pragma once
#include "common.h"

namespace dgs {

// Writes the frame's camera and options to device memory (graph-safe kernel).
void launch_set_frame(hipStream_t st, const FrameK& f, FrameK* dst);

// Neural decode of the cells' Gaussians into planar attribute arrays
// (means [3][M], scales [3][M], raw quaternions [4][M], opacity [M], colour
// [3][M]); cells with cell_ntiles[n] == 0 are skipped (cell_ntiles may be
// null: decode every cell).  weights: the four decoders packed (opacity,
// colour, scale ratio, quaternion), woff[d] = offset of decoder d.
struct DecodeArgs {
    int N, K, F, H;
    const float *cell_pos, *cell_scale, *cell_rot;  // [3][N], [3][N], [4][N]
    const float* features;                          // [F][N]
    const float* offsets;                           // [3][M]
    const float* weights;
    int64_t woff[4];
    const uint32_t* cell_ntiles;
    const FrameK* fr;
    float *means, *scales, *rots, *opac, *color;
};
void launch_decode(hipStream_t st, const DecodeArgs& a);

// offs: CSR member offsets [N+1] (null: the fixed layout) of M Gaussians,
// each cell at most kmax; malformed ranges cull the cell and set
// 1 << kErrInvalid in *err.
void launch_cell_preprocess(hipStream_t st, int N, const float* pos, const float* scale, const float* rot,
                            const float* vsh, int vdeg, const int32_t* offs, int M, int kmax, const FrameK* fr,
                            uint32_t* depth_bits, uint64_t* prect, uint32_t* ntiles, float* v, int* err);

void launch_gauss_project(hipStream_t st, int M, int K, const float* means, const float* scales,
                          const float* rots, const float* opac, const float* sh, int sh_deg, const FrameK* fr,
                          const uint32_t* cell_ntiles, GRec* recs, uint64_t* grect, uint32_t* gdepth,
                          uint32_t* gntiles, bool overlapped = false);

// Exclusive scan of n u32 values (in[i], or in[idx[i]] when idx is set);
// *total receives the sum.  status needs scan_status_words(n) 64-bit words;
// *ticket must be zero; *epoch is the device frame counter (look-back tag
// j = 0).
size_t scan_status_words(int64_t n);
void launch_exclusive_scan(hipStream_t st, const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total,
                           uint64_t* status, const uint32_t* epoch, uint32_t* ticket, int* err,
                           const uint32_t* idx = nullptr);

void launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t v, size_t n);

// Zeroes up to 8 small u32 buffers in one launch (graph-safe: no memset
// nodes) and increments *bump (the look-back frame counter) when set.
struct ClearList {
    uint32_t* p[8];
    size_t n[8];
    int count = 0;
    uint32_t* bump = nullptr;
    void add(uint32_t* ptr, size_t words) {
        p[count] = ptr;
        n[count] = words;
        count++;
    }
};
// With f set, also writes *f to fdst (the frame record) in the same launch.
void launch_clear(hipStream_t st, const ClearList& l, const FrameK* f = nullptr, FrameK* fdst = nullptr);

// Depth sort keys of the primitives: key p = depth bits of p when it touches
// a tile, else all ones (it then sorts last and emits nothing); value = p.
// Also accumulates the four byte histograms of the keys into hist
// ([4][256], zeroed beforehand).
void launch_prim_keys(hipStream_t st, int P, const uint32_t* ntiles, const uint32_t* depth, uint32_t* keys,
                      uint32_t* vals, uint32_t* hist);

// One key per (primitive, touched tile), the primitives taken in depth
// order (order[i], i < P): key = tile << 32 | depth bits, value = primitive
// id, written at offsets[i] in row-major tile order.  A stable sort of these
// keys on the tile bits alone then yields the (tile, depth, id) order.  Also
// accumulates the digit histograms of the kept keys' tile bytes into hist
// ([tile_passes][256], zeroed beforehand).
void launch_emit_keys(hipStream_t st, int P, const uint32_t* order, const uint32_t* ntiles,
                      const uint32_t* offsets, const uint64_t* prect, const uint32_t* depth, int TX, uint32_t cap,
                      uint64_t* keys, uint32_t* vals, uint32_t* hist, int tile_passes, int* err);

// [start, end) per tile of the sorted keys; ranges (2 words per tile) must
// be zero beforehand (tiles without keys keep [0, 0)).  With vout set, the
// sorted values vin are also copied there (a saved frame's own lists).
// Per-tile depth order: each tile's run of the tile-sorted keys (emitted in
// primitive-id order) sorted by (depth bits, id) in place; values also into
// vcopy when set; spare: a free u64 buffer of the key capacity (used by runs
// longer than what one workgroup sorts in registers).  The same launch
// builds the compositor's work queue (as launch_tile_order).
// long_stat, prims: as for launch_tile_order.
void launch_tile_depth_sort(hipStream_t st, const uint32_t* ranges, int tiles, uint64_t* keys, uint32_t* vals,
                            uint64_t* spare, uint32_t* vcopy, uint32_t split_len, uint32_t* order, uint32_t* queue,
                            uint64_t* long_stat = nullptr, uint32_t prims = 0);

// load (nullable, pinned host memory): receives tiles << 32 | key count.
void launch_tile_ranges(hipStream_t st, const uint64_t* keys, const uint32_t* n_ptr, uint32_t cap,
                        uint32_t* ranges, const uint32_t* vin = nullptr, uint32_t* vout = nullptr,
                        uint64_t* load = nullptr, uint32_t tiles = 0);

// Onesweep LSD radix sort of (u64 key, u32 value) pairs on key bits
// [first_bit, first_bit + bits).  The count is read on the device from
// *n_ptr (clamped to cap).  Returns true when the sorted data ends in
// (k1, v1), false for (k0, v0).  hist (8 x 256 words) and tickets (8 words)
// must be zero beforehand; with hist_ready, hist already holds the digit
// counts of the keys (the key emission counts them).  Pass p tags its
// look-back words with epoch_tag(*epoch, tag0 + p).
struct SortScratch {
    uint32_t* hist;     // [passes][256]
    uint64_t* status;   // sort_status_words(cap) look-back words
    uint32_t* tickets;  // [passes]
};
int sort_passes(int bits);
size_t sort_status_words(int64_t cap);
bool launch_radix_sort(hipStream_t st, uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1,
                       const uint32_t* n_ptr, uint32_t cap, int bits, const SortScratch& s,
                       const uint32_t* epoch, int* err, bool hist_ready = false, int first_bit = 0,
                       uint32_t tag0 = 1);
// The same for n (host count) u32 keys on all 32 bits; hist must hold the
// keys' four byte histograms.  Returns true when the data ends in (k1, v1).
bool launch_radix_sort32(hipStream_t st, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n,
                         const SortScratch& s, const uint32_t* epoch, uint32_t tag0, int* err);

struct CompositeArgs {
    const uint32_t* ranges;
    const uint32_t* vals;
    const GRec* recs;
    const float* cell_v;  // Duplex only
    const int32_t* offs;  // [N+1] members of cell n: Gaussians offs[n] .. offs[n+1]-1; null: K per cell
    int K;                // members per cell (fixed), or their upper bound
    const FrameK* fr;  // the frame's camera and options (device)
    CamK k;            // filled from fr inside the kernel
    OptK o;
    float* color;  // the outputs are filled from fr inside the kernel
    float* D;
    float* T;
    int32_t* last;
    unsigned long long* counters;  // [4]: n_val, n_rendered, n_box, n_cell_hits (stats mode), nullable
    uint32_t* order;               // [4 * tiles] scratch: heaviest-first work items
    uint32_t* queue;               // [2] scratch: work-queue head, item count
    bool save;                     // Duplex: also write the frame record's sv_* state (host-side choice)
};
// Work queue of the compositor (costliest-first tile / half-tile items);
// must precede launch_composite_*.  Tiles with at least split_len entries
// become two half-tile items.
// long_stat (nullable, pinned host memory): receives prims << 32 | the
// number of keys in runs of more than 4096 entries.
void launch_tile_order(hipStream_t st, const uint32_t* ranges, int tiles, uint32_t split_len, uint32_t* order,
                       uint32_t* queue, uint64_t* long_stat = nullptr, uint32_t prims = 0);
// Split lengths, measured: lists of cells (each entry K members) and lists
// of Gaussians.
constexpr uint32_t kSplitLenCells = 32;
constexpr uint32_t kSplitLenGauss = 64;
void launch_composite_duplex(hipStream_t st, const CompositeArgs& a);
void launch_composite_alpha(hipStream_t st, const CompositeArgs& a);
// The Duplex walk with LC-WSR cell weights (cell_v holds the weights).
void launch_composite_lcwsr(hipStream_t st, const CompositeArgs& a);

// Backward of the Duplex compositor: per-Gaussian screen-space gradients
// g2d[M][kG2dRow] (row g: mean x, y, conic A, B, C, sigma, r, g, b, then
// padding) and per-cell dL/dv, both accumulated atomically (zero them
// first).  A row fills one 64-byte line, so one member's nine atomics are one
// request.
constexpr int kG2dRow = 16;
struct BwdArgs {
    const uint32_t* ranges;
    const uint32_t* vals;
    const GRec* recs;
    const float* cell_v;
    const int32_t* offs;  // as in CompositeArgs
    int K, M;
    const FrameK* fr;  // the frame's camera and options (device)
    CamK k;            // filled from fr inside the kernels
    OptK o;
    const float* color;
    const float* D;
    const float* T;
    const int32_t* last;
    const float* grad_color;
    const float* grad_D;  // nullable
    float* g2d;
    float* gv;
    uint32_t* order;
    uint32_t* queue;
};
struct ProjBwdArgs {
    int N;
    const float *means, *scales, *rots, *sh;
    int sh_degree;
    const float *cell_pos, *cell_v_sh;
    int v_sh_degree;
    float *d_means, *d_scales, *d_rots, *d_opac, *d_sh, *d_cell_v_sh, *d_cell_pos, *d_mean2d;
    bool overwrite;  // write every entry instead of adding
};
void launch_composite_bwd(hipStream_t st, const BwdArgs& a);
void launch_project_bwd(hipStream_t st, const BwdArgs& a, const ProjBwdArgs& b);

}  // namespace dgs
