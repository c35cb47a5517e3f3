// Internal: the renderer context and entry points shared by the C ABI and
// the serving runtime.
#pragma once
#include <array>
#include <string>
#include <vector>

#include "common.h"
#include "duplexgs.h"
#include "launch.h"

// Text for a device error word with the timeout flag set: which bounded
// look-back wait gave up.
inline std::string timeout_message(int e) {
    std::string m = "device look-back wait timed out in";
    if (e & (1 << dgs::kErrWaitScan)) m += " the exclusive scan";
    if ((e & (1 << dgs::kErrWaitScan)) && (e & (1 << dgs::kErrWaitSort))) m += " and";
    if (e & (1 << dgs::kErrWaitSort)) m += " a radix sort pass";
    return m;
}

// A saved Duplex frame (dgs_render with a non-NULL `saved`): the state its
// backward replays, in buffers of its own so that later renders on the
// context leave it intact.  Released frames stay with their context and are
// reused by later saved renders.
struct dgs_frame_s {
    dgs_ctx owner = nullptr;
    bool live = false;
    dgs::CamK k;  // host copies of the frame's camera and options
    dgs::OptK o;
    int N = 0, K = 0, tiles = 0;
    int64_t M = 0;
    const int32_t* offs = nullptr;  // the scene's CSR offsets (null: fixed layout)
    dgs::GRec* recs = nullptr;  // [M] projected Gaussians
    int64_t cap_recs = 0;
    float* cell_v = nullptr;    // [N] v_n
    int64_t cap_cells = 0;
    uint32_t* vals = nullptr;   // sorted cell ids (the tile lists)
    int64_t cap_vals = 0;
    uint32_t* ranges = nullptr; // [2][tiles] per-tile [start, end)
    uint32_t* order = nullptr;  // [4][tiles] compositor work items
    int64_t cap_tiles = 0;
    float* pix = nullptr;       // [6][H*W]: colour (3 planes), D, replay T, replay start (int32)
    int64_t cap_pix = 0;
    uint32_t* info = nullptr;   // [16]: [0] work-queue head, [1] item count, [2] key total,
                                // [4..13] n_val, n_rendered, n_box, n_cell_hits, n_cell_pixels (u64)
};

struct dgs_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // second stream of the frame: the Gaussian projection runs on it while
    // the cell sort runs on `stream` (fork after the cell preprocess, join
    // before the compositor).  The server turns it off: its slots already
    // overlap whole frames.
    bool two_streams = true;
    int list_order = DGS_LIST_ORDER_AUTO;  // how the tile lists get their depth order
    // The last cell frame's load in pinned host memory (load_dev: its device
    // address), written by the device and read by the next frame's choice of
    // list order: [0] tiles << 32 | keys (0: none yet), as the frame's tile
    // ranges are built; [1] its primitives << 32 | its keys in runs of more
    // than 4096 entries, as its work queue is built.
    uint64_t* load_host = nullptr;
    uint64_t* load_dev = nullptr;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int64_t cap_prims = 0, cap_gauss = 0, cap_keys = 0, cap_tiles = 0;
    uint64_t generation = 0;  // bumped whenever a workspace buffer moves (captured graphs go stale)
    uint32_t *p_depth = nullptr, *p_ntiles = nullptr, *p_offsets = nullptr;
    uint64_t* p_rect = nullptr;
    uint32_t *pk0 = nullptr, *pk1 = nullptr, *pv0 = nullptr, *pv1 = nullptr;  // depth sort of the primitives
    uint64_t* psort_status = nullptr;
    float* cell_v = nullptr;
    dgs::GRec* recs = nullptr;
    uint64_t* grect = nullptr;
    uint64_t *keys0 = nullptr, *keys1 = nullptr;
    uint32_t *vals0 = nullptr, *vals1 = nullptr;
    uint32_t* ranges = nullptr;
    uint32_t* tile_order = nullptr;
    uint64_t* scan_status = nullptr;
    size_t scan_status_cap = 0;
    uint64_t* sort_status = nullptr;
    size_t sort_status_cap = 0;
    dgs::FrameK* frame = nullptr;  // device copy of the current frame's camera and options
    float* dec = nullptr;  // decoded Gaussians of a neural render: [14][M] (means, scales, rots, opacity, colour)
    int64_t cap_dec = 0, dec_gauss = 0;
    bool last_neural = false;
    float* g2d = nullptr;  // [M][kG2dRow] backward screen-space gradients
    float* gv = nullptr;   // [N] backward dL/dv
    int64_t cap_g2d = 0, cap_gv = 0;
    float* loss_coef = nullptr;   // [3][C][H][W] per-pixel coefficients of the loss gradient
    double* loss_part = nullptr;  // [tiles][2] per-tile sums of the loss
    int64_t cap_loss_coef = 0, cap_loss_part = 0;
    uint32_t* hist = nullptr;     // [8][256]: [0..3] primitive depth bytes, [4..6] key tile bytes
    uint32_t* misc = nullptr;     // [0] key total, [1] scan ticket, [2..5] depth sort tickets,
                                  // [6..8] tile sort tickets, [9] spare, [10] sort count,
                                  // [11..12] compositor work-queue head and item count,
                                  // [13] look-back frame counter
    int* dev_err = nullptr;
    unsigned long long* counters = nullptr;  // n_val, n_rendered, n_box, n_cell_hits, n_cell_pixels

    // last frame
    int last_mode = -1, last_passes = 0;
    int64_t last_prims = 0, last_gauss = 0, last_tiles = 0;
    bool last_in_1 = false;

    uint32_t* cur_ranges = nullptr;  // tile ranges of the last render (the context's or a saved frame's)

    // saved frames (live and released), owned by the context
    std::vector<dgs_frame_s*> frames;

    // stage timing
    bool timing = false;
    std::vector<std::array<hipEvent_t, DGS_NUM_STAGES + 1>> events;
    size_t events_used = 0;
};

// Looks up the device address of the static scratch array of
// dgs_sort_pairs_noalloc on `device` (current); once per device.
hipError_t dgs_internal_noalloc_init(int device);

// Workspace capacities (elements): cells or Gaussians that get keys,
// projected Gaussians, sort keys, screen tiles.
struct WorkspaceCaps {
    int64_t prims, gauss, keys, tiles;
};
// Capacities after growing `cur` to hold `want` (the growth policy of every
// render), and the device bytes a context holds at given capacities.
WorkspaceCaps dgs_internal_plan(const WorkspaceCaps& cur, const WorkspaceCaps& want);
int64_t dgs_internal_bytes(const WorkspaceCaps& c);
WorkspaceCaps dgs_internal_caps(dgs_ctx c);
// Key capacity a render starts with when none was reserved.
int64_t dgs_internal_default_keys(int64_t prims);
// Frees the context's workspace (capacities drop to zero); synchronises.
void dgs_internal_release(dgs_ctx c);

// The frame pipeline behind dgs_render.  With write_frame the camera,
// options and output pointers are written to ctx->frame by the first kernel;
// without it the caller has put them there (a captured frame replayed for a
// new camera).  Host-side validation is the same in both cases.
// With nn set, the Gaussians of s are the ones the neural decode writes into
// ctx->dec (sh_degree -1: colour given directly), decoded after cell
// rasterization.
struct NeuralSrc {
    const dgs_neural_scene* scene;
    const dgs_decoder* decoder;
};
// With save set (Duplex only), the frame's replay state goes into *save.
dgs_status dgs_internal_render(dgs_ctx c, const dgs_scene* s, const dgs_camera* cam, const dgs_render_opts* opts,
                               const dgs_image* out, bool write_frame, const NeuralSrc* nn = nullptr,
                               dgs_frame_s* save = nullptr);

// Validates camera, options and output and builds the frame record; *mode
// receives the render mode.  c may be a host-only context (errors land in c->err).
dgs_status dgs_internal_frame(dgs_ctx c, const dgs_camera* cam, const dgs_render_opts* opts, const dgs_image* out,
                              dgs::FrameK* f, int* mode);
dgs_status dgs_internal_check_scene(dgs_ctx c, const dgs_scene* s, int mode);

// Grows the workspace for a render of scene s at width x height with `keys`
// key capacity (allocates and synchronises only when growing).
dgs_status dgs_internal_prepare(dgs_ctx c, const dgs_scene* s, int mode, int width, int height, int64_t keys);
