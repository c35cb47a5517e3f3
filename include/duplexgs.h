/*
 * duplexgs.h -- C ABI of the MI355X (gfx950) Duplex-GS proxy-guided renderer.
 *
 * The renderer implements the per-frame hot path of Duplex-GS (arXiv
 * 2508.03180):
 *   1. cell rasterization (Sec. IV-B): project and near-cull the ellipsoidal
 *      cell proxies (x_n, S_n, Q_n), bound their screen footprint, assign them
 *      to 16x16 tiles and radix-sort one (tile, depth) key per (cell, tile);
 *   2. the hybrid renderer (Sec. V-A, eq. hybrid_renderer, w_n = v_n T_n,
 *      eq. dulpex_T): per pixel, walk the tile's cells front to back, sum each
 *      cell's Gaussians order-free with alpha = sigma G'(x') (eq.
 *      alpha_blending), blend across cells with the cell transmittance and
 *      stop once it falls below eps (Sec. V-B), skipping Gaussians whose
 *      bounding box misses the pixel (Sec. VI-A);
 *   3. as a comparison path in the same library, per-Gaussian keys and
 *      front-to-back alpha blending (eqs. alpha_blending, transmittance).
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers (HIP global memory) unless the
 *     comment says "host".  All floating point data is IEEE binary32.
 *   - Arrays are planar ("component-major"): a [3][N] array stores all x
 *     components, then all y, then all z, each contiguous over N.  This keeps
 *     every per-primitive load coalesced.
 *   - The caller owns scene, image and gradient buffers; the library owns the
 *     context, its workspace and its streams' work.  Nothing is retained past
 *     a call except what the context documents (the last frame's state).
 *   - Every call enqueues work on the context's stream and returns without a
 *     host synchronisation, unless its comment says it synchronises.  A
 *     Duplex frame also runs part of its work (the projection of the cells'
 *     Gaussians) on a second stream the context owns: it starts after the
 *     frame's first kernels on the context's stream and is joined back
 *     before the frame's last kernel there, so the frame is ordered on the
 *     context's stream like a single-stream one (also under graph capture).
 *   - Errors that the host can see return at once and enqueue nothing.
 *     Errors only the device can see (key capacity overflow, a look-back wait
 *     that timed out) set a device flag that dgs_sync / dgs_get_stats report.
 *     Outputs of a failed call are undefined.  Nothing throws across the ABI.
 *   - A context is not thread-safe; use one per host thread / stream.
 */
#ifndef DUPLEXGS_H
#define DUPLEXGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgs_ctx_s* dgs_ctx;
/* Saved forward state of one Duplex frame, for its backward (library-owned,
 * belongs to the context that rendered it). */
typedef struct dgs_frame_s* dgs_frame;

typedef enum {
    DGS_OK = 0,
    DGS_ERR_INVALID_ARG = 1, /* bad pointer, size, degree or camera (also from dgs_sync: bad cell_offsets) */
    DGS_ERR_OOM = 2,         /* device allocation failed */
    DGS_ERR_CAPACITY = 3,    /* more (tile, primitive) keys than reserved; reserve more, render again */
    DGS_ERR_DEVICE = 4,      /* a HIP call failed */
    DGS_ERR_UNSUPPORTED = 5, /* valid request this build does not implement */
    DGS_ERR_TIMEOUT = 6      /* a bounded device-side wait gave up (results invalid) */
} dgs_status;

typedef enum {
    DGS_MODE_DUPLEX = 0, /* per-cell keys + hybrid weighted-sum renderer (Sec. IV-V) */
    DGS_MODE_ALPHA = 1,  /* per-Gaussian keys + sorted alpha blending (comparison path) */
    DGS_MODE_LCWSR = 2   /* the "w/o T^cell" ablation (Sec. VII): the Duplex pipeline with the cell
                            transmittance replaced by the LC-WSR weight (eqs. WSR, LC-WSR) per cell,
                            w_n = v_n max(0, 1 - d_n / lcwsr_tau), d_n the cell's camera depth;
                            C = sum w_n A_n / sum w_n B_n, no termination, final_T = 1 */
} dgs_mode;

#define DGS_FLAG_V_ONE 1u  /* v_n = 1 for every cell (the "w/o v_n" ablation) */
#define DGS_FLAG_NO_ET 2u  /* no early termination (eps = 0) */
#define DGS_FLAG_STATS 4u  /* also count N^val / N^rendered (termination ratio) */

/*
 * Scene (Sec. IV-A): N ellipsoidal cells, each emitting its own Gaussians.
 * Fixed layout (cell_offsets NULL): K per cell, member k of cell n is
 * Gaussian n*K + k, M = N*K.  Ragged layout (cell_offsets set): the members
 * of cell n are Gaussians cell_offsets[n] .. cell_offsets[n+1]-1, at most
 * K of them (a cell may have none), M = num_gaussians.
 */
typedef struct {
    int32_t num_cells;          /* N >= 0 */
    int32_t gaussians_per_cell; /* K in 1..32: members per cell, or with cell_offsets their upper bound */
    const float* cell_pos;      /* [3][N]  x_n */
    const float* cell_scale;    /* [3][N]  S_n, semi-axes (> 0) */
    const float* cell_rot;      /* [4][N]  Q_n as (w, x, y, z); normalised here */
    const float* cell_v_sh;     /* [Cv][N] SH coefficients of logit(v_n), Cv = (v_sh_degree+1)^2 */
    int32_t v_sh_degree;        /* 0..3 */
    const float* means;         /* [3][M]  mu */
    const float* scales;        /* [3][M]  s (> 0) */
    const float* rots;          /* [4][M]  q as (w, x, y, z); normalised here */
    const float* opacities;     /* [M]     sigma in [0, 1]; sigma <= 0 marks an invalid Gaussian */
    const float* sh;            /* [C][3][M] colour SH, C = (sh_degree+1)^2, colour = max(0, 0.5 + sum sh Y) */
    int32_t sh_degree;          /* 0..3 */
    const int32_t* cell_offsets; /* [N+1] device, nullable (fixed layout): CSR offsets, cell_offsets[0] = 0,
                                    non-decreasing, cell_offsets[N] = num_gaussians, each cell's count <= K.
                                    A cell that breaks this is culled and the device error flag set
                                    (DGS_ERR_INVALID_ARG from dgs_sync) */
    int32_t num_gaussians;      /* M of the ragged layout (>= 0); ignored in the fixed layout */
} dgs_scene;

/* Pinhole camera, host struct passed by pointer and copied at the call. */
typedef struct {
    float viewmat[16]; /* row-major world->camera [R | t; 0 0 0 1], OpenCV axes (x right, y down, z forward) */
    float fx, fy, cx, cy;
    int32_t width, height; /* 1..32767 */
    float z_near;          /* primitives with camera depth <= z_near are culled */
} dgs_camera;

/* Render options, host struct.  dgs_default_opts fills the defaults. */
typedef struct {
    int32_t mode;          /* dgs_mode */
    uint32_t flags;        /* DGS_FLAG_* */
    float eps_T;           /* termination threshold on the transmittance in front of a cell (1e-4) */
    float alpha_min;       /* alpha below this is skipped (1/255) */
    float alpha_max;       /* alpha clamp (0.99); must lie in (0, 1), so every factor 1 - v alpha > 0 */
    float cov2d_dilation;  /* screen-space variance added to every Gaussian, px^2 (0.3) */
    float proxy_kappa;     /* cell footprint = kappa-sigma box of the projected proxy (1.0) */
    float bg[3];           /* colour of pixels no Gaussian reaches (0, 0, 0) */
    float lcwsr_tau;       /* DGS_MODE_LCWSR only: the depth where the weight reaches 0 (> 0; default 0) */
} dgs_render_opts;

/* Output image, caller-owned device buffers, row-major. */
typedef struct {
    float* color;      /* [3][H][W] */
    float* weight_sum; /* [H][W] D = sum_n w_n sum_k alpha (Duplex) or 1 - T (alpha), nullable */
    float* final_T;    /* [H][W] transmittance behind the last blended cell, nullable */
    int32_t* last;     /* [H][W] 1 + tile-list position of the last contributing entry (0 = none): the
                          last cell (Gaussian in alpha mode) with a member that passed the box and
                          alpha_min gates at the pixel, whatever its weight v_n; nullable */
} dgs_image;

/* Gradients: caller-owned device buffers in the scene's planar layout.  With
 * overwrite == 0 the library ADDS into them (zero them first, or accumulate
 * over several frames); with overwrite != 0 it writes every entry of every
 * buffer (zero where there is no gradient), so they need no clearing and are
 * not read.  Cell scales and rotations only
 * decide which tiles a cell is listed in (a discrete choice), so they get no
 * gradient; cell positions get the gradient through the view direction of
 * v_n only. */
typedef struct {
    float* d_means;     /* [3][M] */
    float* d_scales;    /* [3][M] */
    float* d_rots;      /* [4][M] (w, x, y, z) */
    float* d_opacities; /* [M] */
    float* d_sh;        /* [C][3][M] */
    float* d_cell_v_sh; /* [Cv][N] */
    float* d_cell_pos;  /* [3][N] */
    float* d_mean2d;    /* [2][M] gradient of the projected means (densification statistics), nullable */
    int32_t overwrite;  /* 0: add into the buffers; nonzero: write them */
} dgs_grads;

typedef struct {
    int64_t num_keys;      /* (tile, primitive) keys of the last render */
    int64_t key_capacity;  /* reserved key capacity */
    int64_t n_val;         /* sum over pixels of N^val (DGS_FLAG_STATS renders only) */
    int64_t n_rendered;    /* sum over pixels of N^rendered (DGS_FLAG_STATS renders only) */
    int64_t n_box;         /* (pixel, Gaussian) pairs evaluated inside the Gaussian's box before termination */
    int64_t n_cell_hits;   /* (pixel, list entry) pairs that contributed (Duplex: cells; alpha: Gaussians) */
    int32_t device_error;  /* dgs_status of the last device-side error, 0 if none */
    int32_t sort_passes;   /* radix passes of the last sort */
    int64_t n_cell_pixels; /* (pixel, cell) pairs the cell walks reach (listed cells of the pixel's tile before
                              termination; DGS_FLAG_STATS renders in the Duplex and LC-WSR modes, else 0) */
} dgs_stats;

/* Fills *opts with the defaults listed above (mode Duplex, flags 0). */
void dgs_default_opts(dgs_render_opts* opts);

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle. */
dgs_status dgs_create(int device, void* hip_stream, dgs_ctx* out);

/* Waits for the context's work and frees everything it owns. */
dgs_status dgs_destroy(dgs_ctx ctx);

/* Changes the stream later calls enqueue on. */
dgs_status dgs_set_stream(dgs_ctx ctx, void* hip_stream);

/* Overlap inside a frame (on by default): a Duplex or LC-WSR frame projects
 * its members (Sec. IV-A, the Gaussians each cell emits) on a second stream
 * of the context while the cells are sorted (Sec. IV-B), and joins it
 * before compositing.  The second stream is created by the first frame that
 * uses it (never inside a graph capture: such a frame runs on one stream).
 * Callers that overlap whole frames themselves -- several contexts on
 * several streams -- can turn it off (enable = 0) so that each context
 * holds one stream.  Results are identical either way. */
dgs_status dgs_set_overlap(dgs_ctx ctx, int32_t enable);

/* How a frame puts each tile's list in depth order (Sec. IV-B: the keys are
 * sorted by tile, then by depth; ties by primitive id).  Both ways give the
 * same lists bit for bit:
 *   DGS_LIST_ORDER_GLOBAL: the primitives (cells, or Gaussians in
 *     DGS_MODE_ALPHA) are radix-sorted by depth first and their keys emitted
 *     in that order, then stably sorted on the tile bits;
 *   DGS_LIST_ORDER_PER_TILE: the keys are emitted in primitive-id order,
 *     stably sorted on the tile bits, and each tile's run is then sorted by
 *     (depth, id) on its own (fast when the lists are short);
 *   DGS_LIST_ORDER_AUTO (default): per tile for per-cell lists (Duplex,
 *     LC-WSR) when the context's last such frame had at most 8 keys per
 *     cell, at most 1024 keys per screen tile on
 *     average and at most a twentieth of its keys in tile runs of more than
 *     4096 entries (the device leaves those counts in pinned host memory as the
 *     frame's lists are built; before any such frame: when the key capacity
 *     is at most 256 keys per tile), else global (always for
 *     DGS_MODE_ALPHA).
 * The setting holds for the context's later frames; it changes no result.
 * Other values: DGS_ERR_INVALID_ARG. */
enum { DGS_LIST_ORDER_AUTO = 0, DGS_LIST_ORDER_PER_TILE = 1, DGS_LIST_ORDER_GLOBAL = 2 };
dgs_status dgs_set_list_order(dgs_ctx ctx, int32_t order);

/* Sizes the workspace for up to max_keys (tile, primitive) keys,
 * max_prims cells or Gaussians and max_tiles screen tiles.  Allocates (and
 * synchronises) only when growing.  Render grows prims/tiles by itself;
 * the key capacity only grows here, so call it before graph capture. */
dgs_status dgs_reserve(dgs_ctx ctx, int64_t max_keys, int64_t max_prims, int64_t max_tiles);

/* Renders one frame: all of Sec. IV-B, V-A, V-B and VI-A for DGS_MODE_DUPLEX,
 * per-Gaussian alpha blending for DGS_MODE_ALPHA.  opts may be NULL
 * (defaults).  The context keeps this frame's sorted lists and discrete
 * results until its next render (the dgs_read_* calls).
 *
 * saved (nullable): for a frame that will be differentiated.  When non-NULL
 * (DGS_MODE_DUPLEX only, else DGS_ERR_UNSUPPORTED), *saved receives a frame
 * handle holding everything dgs_render_backward replays -- the per-tile cell
 * lists, the projected Gaussians, v_n, and per pixel the colour, D and the
 * transmittance at the replay start -- in buffers of its own: later renders,
 * dgs_reserve and dgs_sort_pairs on the context leave it intact, so several
 * frames can await their backward on one context.  It stays valid until
 * dgs_frame_release or dgs_destroy.  A saved render may allocate device
 * memory (not for graph capture). */
dgs_status dgs_render(dgs_ctx ctx, const dgs_scene* scene, const dgs_camera* cam, const dgs_render_opts* opts,
                      const dgs_image* out, dgs_frame* saved);

/* Backward of the hybrid renderer (Sec. V-A eqs. hybrid_renderer and
 * dulpex_T, with w_n = v_n T_n): given dL/dC (grad_color, [3][H][W]) and
 * optionally dL/dD (grad_weight_sum, [H][W], nullable), adds dL/d(parameters)
 * into *grads (or writes them, see dgs_grads.overwrite).  It replays the
 * saved frame `saved`, which must come from dgs_render on this context with
 * the same scene arrays (same sizes; their values must not have changed since).
 * cam and opts may be NULL (the frame's own); when given they must equal the
 * frame's, else DGS_ERR_INVALID_ARG.  The transmittance in front of each cell
 * is recovered back to front from the one stored at the replay start, so no
 * division meets a vanishing factor; cells whose front transmittance is below
 * 2^-64 (reachable only with termination off or eps below that) get no
 * gradient.  Gradients are summed with float atomics, so their last bits may
 * differ between runs.  The frame stays valid (a second backward of it is
 * allowed). */
dgs_status dgs_render_backward(dgs_ctx ctx, const dgs_scene* scene, const dgs_camera* cam,
                               const dgs_render_opts* opts, dgs_frame saved, const float* grad_color,
                               const float* grad_weight_sum, const dgs_grads* grads);

/* Gives a saved frame back to its context (stream-ordered: work already
 * enqueued on the context's stream that reads it still sees it).  The
 * handle is invalid afterwards. */
dgs_status dgs_frame_release(dgs_ctx ctx, dgs_frame saved);



/* Waits for the context's stream; returns the first device-side error since
 * the previous dgs_sync (DGS_ERR_CAPACITY, DGS_ERR_TIMEOUT) or DGS_OK. */
dgs_status dgs_sync(dgs_ctx ctx);

/* Synchronises and reports the counters of the last render. */
dgs_status dgs_get_stats(dgs_ctx ctx, dgs_stats* out);

/* Synchronises and reports the counters of a saved frame's render
 * (num_keys, key_capacity and, for DGS_FLAG_STATS renders, n_val, n_rendered,
 * n_box and n_cell_hits; the termination ratio is 1 - n_rendered / n_val). */
dgs_status dgs_frame_stats(dgs_ctx ctx, dgs_frame saved, dgs_stats* out);

/* Message of the last host-side error of this context (never NULL). */
const char* dgs_last_error(dgs_ctx ctx);

/* Introspection of the last render, for parity checks and tools.
 * Copies (asynchronously) the sorted keys (u64: tile << 32 | depth bits),
 * sorted values (u32 primitive ids) and per-tile [start, end) ranges (u32
 * pairs) into caller buffers; any pointer may be NULL.  Buffers must hold
 * num_keys / num_keys / 2*tiles entries (num_keys from dgs_get_stats). */
dgs_status dgs_read_lists(dgs_ctx ctx, uint64_t* keys, uint32_t* values, uint32_t* ranges);

/* Copies per-primitive discrete results of the last render: for cells
 * (Duplex) or Gaussians (alpha mode), the inclusive pixel rectangle
 * x0,x1,y0,y1 as int32 [P][4] (-1 when culled), the depth key bits [P] and
 * the tile count [P].  Any pointer may be NULL. */
dgs_status dgs_read_prims(dgs_ctx ctx, int32_t* rect, uint32_t* depth_bits, uint32_t* ntiles);

/* Copies the inclusive pixel rectangles of all M Gaussians of the last
 * render ([M][4] int32, -1 when culled or not projected). */
dgs_status dgs_read_gauss_rects(dgs_ctx ctx, int32_t* rect);

/*
 * Neural scenes (Sec. III-A neural Gaussians with the cell proxy of
 * Sec. IV-A): each cell carries a latent feature f_n and emits K Gaussians
 * whose attributes four shared two-layer MLPs decode from (f_n, delta_n,
 * d_n), delta_n / d_n the distance / unit direction from the camera centre
 * to x_n.  Each decoder is Linear(F+4 -> H), ReLU, Linear(H -> K a) with
 *   d = 0  opacity       a = 1  sigma = tanh(y) (a Gaussian is valid iff sigma > 0)
 *   d = 1  colour        a = 3  c = sigmoid(y)
 *   d = 2  scale ratio   a = 3  r = max(0, min(sigmoid(y), 1 - |O^pos|)), s = r * S_n
 *                               (eqs. nerual_scales, scale_res)
 *   d = 3  quaternion    a = 4  q = y (normalised where used)
 * and centres mu = x_n + R(Q_n)(O^pos * S_n) (eq. scaffold_offset, the
 * offset O^pos in the cell frame).  Output o of decoder d belongs to member
 * o / a, component o % a.  Only cells that pass cell rasterization are
 * decoded (every cell in DGS_MODE_ALPHA).
 */
typedef struct {
    int32_t feature_dim;   /* F in 1..64 */
    int32_t hidden_dim;    /* H in 1..64 */
    const float* weights;  /* device; for d = 0..3 in order: W1[(F+4)][H] (input-major: W1[i*H + j]),
                              b1[H], W2[H][K a] (W2[j*K*a + o]), b2[K a]; input order
                              (f_0 .. f_{F-1}, delta, d_x, d_y, d_z) */
} dgs_decoder;

typedef struct {
    int32_t num_cells;          /* N >= 0 */
    int32_t gaussians_per_cell; /* K in 1..32 */
    const float* cell_pos;      /* [3][N] */
    const float* cell_scale;    /* [3][N] */
    const float* cell_rot;      /* [4][N] */
    const float* cell_v_sh;     /* [Cv][N] */
    int32_t v_sh_degree;        /* 0..3 */
    const float* features;      /* [F][N] latent features */
    const float* offsets;       /* [3][M] O^pos per Gaussian, |O^pos| <= 1 expected */
} dgs_neural_scene;

/* Renders a neural scene: cell rasterization, decode of the visible cells'
 * Gaussians, then the same pipeline as dgs_render (DGS_MODE_DUPLEX,
 * DGS_MODE_LCWSR or DGS_MODE_ALPHA).  The decoded attributes stay in the
 * context's workspace until the next render (dgs_read_decoded).  No
 * backward. */
dgs_status dgs_render_neural(dgs_ctx ctx, const dgs_neural_scene* scene, const dgs_decoder* decoder,
                             const dgs_camera* cam, const dgs_render_opts* opts, const dgs_image* out);

/* Copies (asynchronously) the Gaussians decoded by the last
 * dgs_render_neural into caller device buffers, planar: means [3][M],
 * scales [3][M], raw quaternions [4][M], opacities [M], colours [3][M]; any
 * pointer may be NULL.  Entries of cells that were not decoded are
 * undefined. */
dgs_status dgs_read_decoded(dgs_ctx ctx, float* means, float* scales, float* rots, float* opacities, float* colors);

/* Stage timing.  While enabled, every render records HIP events on the
 * context stream at the boundaries of its stages (and runs all of a frame on
 * that stream, so the stages do not overlap):
 *   0 cell preprocess (or nothing in alpha mode), 1 Gaussian projection,
 *   2 depth sort of the primitives (empty with the per-tile list order),
 *   3 scan + key emission, 4 radix sort of the keys on their tile bits,
 *   5 tile ranges, 6 per-tile depth order (empty with the global list
 *   order; it also builds the compositor's work queue), 7 compositor work
 *   queue (empty with the per-tile list order), 8 the compositor kernel
 *   alone. */
#define DGS_NUM_STAGES 9
dgs_status dgs_set_timing(dgs_ctx ctx, int32_t enable);

/* Synchronises; writes the summed milliseconds of each stage over the renders
 * timed since the previous call into ms[0..n_stages-1] (host array) and their
 * number into *frames (host), then starts a new tally. */
dgs_status dgs_get_timing(dgs_ctx ctx, float* ms, int32_t n_stages, int32_t* frames);

/* Stable in-place sort of n (key, value) pairs on the low key_bits bits
 * (1..64) with the library's onesweep radix sort.  keys/values are device
 * buffers of n entries. */
dgs_status dgs_sort_pairs(dgs_ctx ctx, uint64_t* keys, uint32_t* values, int64_t n, int32_t key_bits);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sort as dgs_sort_pairs, with the same results, whose scratch memory (the
 * ping-pong key/value buffers, digit counts, look-back words and counters,
 * ~14.3 MB) is one static device array per GPU, held from library load until
 * the process ends.  It calls no hipMalloc, hipFree or allocating routine;
 * it enqueues on the context's stream (kernels and device-to-device copies,
 * no memset).  n above DGS_SORT_NOALLOC_MAX_KEYS returns DGS_ERR_INVALID_ARG
 * and enqueues nothing.  All calls on one GPU share that GPU's array, from
 * every context and thread: calls whose work overlaps on one GPU (different
 * streams, or threads) race and give undefined results; serialise them.
 * Device-side errors (a look-back wait that timed out) are reported by
 * dgs_sync on the context. */
#define DGS_SORT_NOALLOC_MAX_KEYS (1 << 20)
dgs_status dgs_sort_pairs_noalloc(dgs_ctx ctx, uint64_t* keys, uint32_t* values, int64_t n, int32_t key_bits);

/*
 * Training loss (eq. `loss`, Sec. "Perceptual Loss"; lambda_1 = 0.2 in Sec.
 * "Experimental Settings") without its perceptual term:
 *     L = (1 - lambda) mean |image - target| + lambda (1 - mean SSIM),
 * the means over every channel and pixel; SSIM per channel from an 11 x 11
 * Gaussian window (sigma 1.5, weights summing to 1), the images zero
 * outside their borders, c1 = 0.01^2, c2 = 0.03^2.
 * image, target: device, planar [channels][height][width] binary32.
 * loss: device, one float, written on the context's stream (no host
 * synchronisation).  grad_image: device [channels][height][width], dL/dimage
 * written whole (0 from the l1 term where image == target), or NULL for the
 * loss alone.  The per-pixel gradient coefficients live in the context's
 * workspace (3 floats per pixel, grown on demand).  The sum is taken in a
 * fixed order, so repeated calls give identical results.
 * Errors: DGS_ERR_INVALID_ARG for a NULL pointer, sizes outside 1..32767
 * (channels 1..65535) or lambda outside [0, 1]; DGS_ERR_OOM when the
 * workspace cannot grow.
 */
dgs_status dgs_loss_l1_ssim(dgs_ctx ctx, const float* image, const float* target, int32_t channels,
                            int32_t height, int32_t width, float lambda, float* loss, float* grad_image);

/*
 * Serving runtime.  A server renders requests (scene, camera, options,
 * output image) submitted from any host thread.  It keeps num_slots frames
 * in flight, each slot with its own context, workspace and HIP stream, and
 * starts the next queued request as soon as a slot frees (continuous
 * batching).  Requests start in submission order; one whose workspace would
 * push the slots' total over memory_budget waits until running frames finish
 * (idle slots give their workspace back first), and one that could not fit
 * even alone fails with DGS_ERR_OOM.  With use_graphs, the first request of
 * each (scene, image size, mode, DGS_FLAG_STATS) on a slot is captured into a
 * HIP graph and later ones replay it with their own camera, options and
 * output pointers.  A frame that overflows its key capacity is run again
 * after the slot grows (up to 4 attempts).  Results are bit-identical to
 * dgs_render of the same request.  Every server function is thread-safe.
 * Scene arrays and output buffers are caller-owned device memory that must
 * stay valid until the requests using them have finished.
 */
typedef struct dgs_server_s* dgs_server;

typedef struct {
    int32_t num_slots;     /* frames in flight (1..16); each holds its own workspace */
    int32_t use_graphs;    /* nonzero: capture and replay HIP graphs per request shape */
    int64_t memory_budget; /* bytes of workspace all slots may hold together; 0 = unlimited */
} dgs_server_config;

/* Host-only stand-in for the device, for tests of the scheduler: a frame
 * takes seconds_fixed + seconds_per_mpixel * W*H/1e6 seconds and produces
 * keys_per_pixel * W*H keys (more than the slot's capacity is an overflow).
 * Workspace is accounted exactly as on the device but nothing is allocated
 * and no pointer is dereferenced. */
typedef struct {
    double seconds_fixed;
    double seconds_per_mpixel;
    double keys_per_pixel;
} dgs_sim_device;

typedef enum {
    DGS_REQ_QUEUED = 0,
    DGS_REQ_RUNNING = 1,
    DGS_REQ_DONE = 2,      /* output written */
    DGS_REQ_FAILED = 3,    /* result holds the dgs_status */
    DGS_REQ_CANCELLED = 4
} dgs_request_state;

typedef struct {
    int32_t state;    /* dgs_request_state */
    int32_t result;   /* dgs_status of a finished request */
    int32_t slot;     /* slot of the last attempt (-1 before the first) */
    int32_t attempts; /* launches, including capacity retries */
    int32_t graph;    /* last attempt: 0 direct launches, 1 graph replay, 2 graph captured */
    int32_t reserved;
    int64_t num_keys; /* (tile, primitive) keys of the last attempt */
    double t_submit;  /* host steady-clock seconds: submission, first launch, completion seen */
    double t_start;
    double t_done;
} dgs_request_info;

typedef struct {
    int64_t submitted, completed, failed, cancelled;
    int64_t retries;        /* capacity-overflow re-runs */
    int64_t graph_captures, graph_replays;
    int64_t releases;       /* idle workspaces given back for the memory budget */
    int64_t workspace_bytes, peak_workspace_bytes;
    int64_t queued, running;
} dgs_server_stats;

/* num_slots 4, use_graphs 1, memory_budget 0. */
void dgs_server_default_config(dgs_server_config* cfg);
dgs_status dgs_server_create(int device, const dgs_server_config* cfg, dgs_server* out);
dgs_status dgs_server_create_simulated(const dgs_server_config* cfg, const dgs_sim_device* sim, dgs_server* out);
/* Registers a scene (device arrays, caller-owned); *scene_id receives its id. */
dgs_status dgs_server_add_scene(dgs_server srv, const dgs_scene* scene, int32_t* scene_id);
/* Validates and queues a request (host structs are copied; opts may be
 * NULL); *request_id receives its id.  Returns at once. */
dgs_status dgs_server_submit(dgs_server srv, int32_t scene_id, const dgs_camera* cam, const dgs_render_opts* opts,
                             const dgs_image* out, int64_t* request_id);
/* Current state of a request (host struct). */
dgs_status dgs_server_query(dgs_server srv, int64_t request_id, dgs_request_info* info);
/* Blocks until the request has finished (timeout_s < 0: no limit);
 * DGS_ERR_TIMEOUT if it has not within timeout_s.  info may be NULL. */
dgs_status dgs_server_wait(dgs_server srv, int64_t request_id, double timeout_s, dgs_request_info* info);
/* Cancels a request that has not started (DGS_ERR_INVALID_ARG otherwise). */
dgs_status dgs_server_cancel(dgs_server srv, int64_t request_id);
/* Forgets a finished request. */
dgs_status dgs_server_release(dgs_server srv, int64_t request_id);
dgs_status dgs_server_get_stats(dgs_server srv, dgs_server_stats* out);
/* Message of the server's last error (never NULL; valid until the calling
 * thread's next call of this function). */
const char* dgs_server_last_error(dgs_server srv);
/* Cancels queued requests, waits for running ones and frees everything. */
dgs_status dgs_server_destroy(dgs_server srv);

#ifdef __cplusplus
}
#endif
#endif /* DUPLEXGS_H */
