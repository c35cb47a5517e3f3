// C ABI of the renderer: context, workspace and the per-frame pipeline.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <vector>

#include "ctx.h"

using namespace dgs;



namespace {

dgs_status fail(dgs_ctx c, dgs_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

template <class T>
hipError_t grow(T*& p, int64_t want, hipStream_t st) {
    if (p) {
        hipStreamSynchronize(st);
        hipFree(p);
        p = nullptr;
    }
    return hipMalloc((void**)&p, sizeof(T) * (size_t)(want > 0 ? want : 1));
}

// Look-back status buffers start zeroed (epoch 0 is never used).  The
// zeroing is a fill kernel on the context's stream, ordered before the
// frames that use the buffer: a null-stream memset is not ordered with a
// non-blocking stream and could erase status words in the middle of a sort.
hipError_t grow_zeroed(uint64_t*& p, int64_t want, hipStream_t st) {
    hipError_t e = grow(p, want, st);
    if (e == hipSuccess) {
        launch_fill_u32(st, reinterpret_cast<uint32_t*>(p), 0u, 2 * (size_t)(want > 0 ? want : 1));
        e = hipGetLastError();
    }
    return e;
}

dgs_status ensure(dgs_ctx c, int64_t prims, int64_t gauss, int64_t keys, int64_t tiles) {
    if (keys > (int64_t)(1u << 30)) return fail(c, DGS_ERR_INVALID_ARG, "key capacity above 2^30");
    const WorkspaceCaps cur{c->cap_prims, c->cap_gauss, c->cap_keys, c->cap_tiles};
    const WorkspaceCaps nc = dgs_internal_plan(cur, WorkspaceCaps{prims, gauss, keys, tiles});
    hipError_t e = hipSuccess;
    if (nc.prims != cur.prims) {
        c->generation++;
        if ((e = grow(c->p_depth, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->p_ntiles, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->p_offsets, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->p_rect, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->cell_v, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->pk0, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->pk1, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->pv0, nc.prims, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->pv1, nc.prims, c->stream)) != hipSuccess) goto oom;
        size_t sw = scan_status_words(nc.prims);
        if ((e = grow_zeroed(c->scan_status, (int64_t)sw, c->stream)) != hipSuccess) goto oom;
        c->scan_status_cap = sw;
        if ((e = grow_zeroed(c->psort_status, (int64_t)sort_status_words(nc.prims), c->stream)) != hipSuccess)
            goto oom;
        c->cap_prims = nc.prims;
    }
    if (nc.gauss != cur.gauss) {
        c->generation++;
        if ((e = grow(c->recs, nc.gauss, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->grect, nc.gauss, c->stream)) != hipSuccess) goto oom;
        c->cap_gauss = nc.gauss;
    }
    if (nc.keys != cur.keys) {
        c->generation++;
        if ((e = grow(c->keys0, nc.keys, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->keys1, nc.keys, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->vals0, nc.keys, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->vals1, nc.keys, c->stream)) != hipSuccess) goto oom;
        size_t sw = sort_status_words(nc.keys);
        if ((e = grow_zeroed(c->sort_status, (int64_t)sw, c->stream)) != hipSuccess) goto oom;
        c->sort_status_cap = sw;
        c->cap_keys = nc.keys;
    }
    if (nc.tiles != cur.tiles) {
        c->generation++;
        if ((e = grow(c->ranges, 2 * nc.tiles, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(c->tile_order, 4 * nc.tiles, c->stream)) != hipSuccess) goto oom;
        c->cap_tiles = nc.tiles;
    }
    if (nc.prims != cur.prims || nc.gauss != cur.gauss || nc.keys != cur.keys || nc.tiles != cur.tiles) {
        // the last render's lists and discrete results are gone (saved frames keep their own)
        c->last_mode = -1;
        c->cur_ranges = nullptr;
    }
    return DGS_OK;
oom:
    // a partial growth leaves the buffers of the failed group unusable: drop them all
    dgs_internal_release(c);
    return fail(c, DGS_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
}

bool finite_f(float x) { return x == x && x > -INFINITY && x < INFINITY; }

dgs_status make_cam(dgs_ctx c, const dgs_camera* cam, CamK& k) {
    if (!cam) return fail(c, DGS_ERR_INVALID_ARG, "camera is NULL");
    if (cam->width < 1 || cam->height < 1 || cam->width > 32767 || cam->height > 32767)
        return fail(c, DGS_ERR_INVALID_ARG, "image size must be in 1..32767");
    for (int i = 0; i < 16; i++)
        if (!finite_f(cam->viewmat[i])) return fail(c, DGS_ERR_INVALID_ARG, "viewmat is not finite");
    if (!(cam->fx > 0) || !(cam->fy > 0) || !finite_f(cam->fx) || !finite_f(cam->fy) || !finite_f(cam->cx) ||
        !finite_f(cam->cy))
        return fail(c, DGS_ERR_INVALID_ARG, "focal lengths must be finite and > 0");
    if (!(cam->z_near > 0) || !finite_f(cam->z_near)) return fail(c, DGS_ERR_INVALID_ARG, "z_near must be > 0");
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) {
            k.R[i * 3 + j] = cam->viewmat[i * 4 + j];
            k.Rd[i * 3 + j] = cam->viewmat[i * 4 + j];
        }
        k.t[i] = cam->viewmat[i * 4 + 3];
        k.td[i] = cam->viewmat[i * 4 + 3];
    }
    for (int j = 0; j < 3; j++)
        k.o[j] = (float)(-(k.Rd[0 * 3 + j] * k.td[0] + k.Rd[1 * 3 + j] * k.td[1] + k.Rd[2 * 3 + j] * k.td[2]));
    k.fx = cam->fx; k.fy = cam->fy; k.cx = cam->cx; k.cy = cam->cy;
    k.znear = cam->z_near;
    k.W = cam->width; k.H = cam->height;
    k.TX = (k.W + kTile - 1) / kTile;
    k.TY = (k.H + kTile - 1) / kTile;
    return DGS_OK;
}

dgs_status make_opts(dgs_ctx c, const dgs_render_opts* in, OptK& o, int& mode) {
    dgs_render_opts d;
    dgs_default_opts(&d);
    const dgs_render_opts& p = in ? *in : d;
    if (p.mode != DGS_MODE_DUPLEX && p.mode != DGS_MODE_ALPHA && p.mode != DGS_MODE_LCWSR)
        return fail(c, DGS_ERR_INVALID_ARG, "unknown mode");
    if (p.mode == DGS_MODE_LCWSR && !(p.lcwsr_tau > 0 && finite_f(p.lcwsr_tau)))
        return fail(c, DGS_ERR_INVALID_ARG, "DGS_MODE_LCWSR needs a finite lcwsr_tau > 0");
    if (!(p.alpha_min > 0) || !(p.alpha_max > 0) || !(p.alpha_max < 1.0f) || !(p.eps_T >= 0) ||
        !(p.cov2d_dilation >= 0) || !(p.proxy_kappa > 0))
        return fail(c, DGS_ERR_INVALID_ARG, "render options out of range");
    mode = p.mode;
    o.eps = p.eps_T;
    o.alpha_max = p.alpha_max;
    o.log2_alpha_min = log2f(p.alpha_min);
    o.delta = p.cov2d_dilation;
    o.kappa = p.proxy_kappa;
    for (int i = 0; i < 3; i++) o.bg[i] = p.bg[i];
    o.v_one = (p.flags & DGS_FLAG_V_ONE) != 0;
    o.no_et = (p.flags & DGS_FLAG_NO_ET) != 0;
    o.stats = (p.flags & DGS_FLAG_STATS) != 0;
    o.tau = p.mode == DGS_MODE_LCWSR ? p.lcwsr_tau : 0.0f;
    return DGS_OK;
}

// Number of Gaussians of a scene (fixed or ragged layout).
int64_t scene_gaussians(const dgs_scene* s) {
    return s->cell_offsets ? (int64_t)s->num_gaussians : (int64_t)s->num_cells * s->gaussians_per_cell;
}

dgs_status check_scene(dgs_ctx c, const dgs_scene* s, int mode, bool decoded = false) {
    if (!s) return fail(c, DGS_ERR_INVALID_ARG, "scene is NULL");
    if (s->num_cells < 0) return fail(c, DGS_ERR_INVALID_ARG, "num_cells < 0");
    if (s->gaussians_per_cell < 1 || s->gaussians_per_cell > kMaxK)
        return fail(c, DGS_ERR_INVALID_ARG, "gaussians_per_cell must be in 1..32");
    if (s->cell_offsets && s->num_gaussians < 0) return fail(c, DGS_ERR_INVALID_ARG, "num_gaussians < 0");
    if (scene_gaussians(s) > (int64_t)(1 << 30)) return fail(c, DGS_ERR_INVALID_ARG, "too many Gaussians");
    if (s->sh_degree < (decoded ? -1 : 0) || s->sh_degree > 3 || s->v_sh_degree < 0 || s->v_sh_degree > 3)
        return fail(c, DGS_ERR_INVALID_ARG, "SH degree must be in 0..3");
    if (s->num_cells == 0) return DGS_OK;
    if (scene_gaussians(s) > 0 && (!s->means || !s->scales || !s->rots || !s->opacities || !s->sh))
        return fail(c, DGS_ERR_INVALID_ARG, "Gaussian arrays must not be NULL");
    if (mode != DGS_MODE_ALPHA && (!s->cell_pos || !s->cell_scale || !s->cell_rot || !s->cell_v_sh))
        return fail(c, DGS_ERR_INVALID_ARG, "cell arrays must not be NULL");
    return DGS_OK;
}

int tile_bits(int tiles) {
    int b = 0;
    while ((1 << b) < tiles) b++;
    return b;
}

dgs_status launched(dgs_ctx c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, DGS_ERR_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    return DGS_OK;
}

// Event marking the start of stage `i` (i == DGS_NUM_STAGES: end of frame).
struct StageMarks {
    dgs_ctx c;
    std::array<hipEvent_t, DGS_NUM_STAGES + 1>* ev = nullptr;
    explicit StageMarks(dgs_ctx ctx) : c(ctx) {
        if (!c->timing) return;
        if (c->events_used == c->events.size()) {
            std::array<hipEvent_t, DGS_NUM_STAGES + 1> a;
            for (auto& e : a) hipEventCreate(&e);
            c->events.push_back(a);
        }
        ev = &c->events[c->events_used++];
    }
    void mark(int i) {
        if (ev) hipEventRecord((*ev)[i], c->stream);
    }
};

__global__ void k_unpack_rects(const uint64_t* in, int64_t n, int32_t* out) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t r = in[i];
    if (r == kEmptyRect) {
        out[4 * i] = out[4 * i + 1] = out[4 * i + 2] = out[4 * i + 3] = -1;
    } else {
        out[4 * i] = rect_x0(r); out[4 * i + 1] = rect_x1(r);
        out[4 * i + 2] = rect_y0(r); out[4 * i + 3] = rect_y1(r);
    }
}

int64_t decoder_floats(int F, int H, int K, int64_t* woff) {
    static const int A[4] = {1, 3, 3, 4};
    int64_t n = 0;
    for (int d = 0; d < 4; d++) {
        if (woff) woff[d] = n;
        n += (int64_t)(F + 4) * H + H + (int64_t)H * K * A[d] + (int64_t)K * A[d];
    }
    return n;
}

DecodeArgs decode_args(dgs_ctx c, const NeuralSrc& nn, const uint32_t* cell_ntiles) {
    const dgs_neural_scene& s = *nn.scene;
    DecodeArgs a;
    a.N = s.num_cells;
    a.K = s.gaussians_per_cell;
    a.F = nn.decoder->feature_dim;
    a.H = nn.decoder->hidden_dim;
    a.cell_pos = s.cell_pos;
    a.cell_scale = s.cell_scale;
    a.cell_rot = s.cell_rot;
    a.features = s.features;
    a.offsets = s.offsets;
    a.weights = nn.decoder->weights;
    decoder_floats(a.F, a.H, a.K, a.woff);
    a.cell_ntiles = cell_ntiles;
    a.fr = c->frame;
    const int64_t M = (int64_t)a.N * a.K;
    a.means = c->dec;
    a.scales = c->dec + 3 * M;
    a.rots = c->dec + 6 * M;
    a.opac = c->dec + 10 * M;
    a.color = c->dec + 11 * M;
    return a;
}

void free_frame(dgs_frame_s* f) {
    void* ptrs[] = {f->recs, f->cell_v, f->vals, f->ranges, f->order, f->pix, f->info};
    for (void* p : ptrs)
        if (p) hipFree(p);
    delete f;
}

// A released frame of the context (or a new one) with room for a render of
// N cells, M Gaussians, `keys` keys, `tiles` tiles and `pixels` pixels.
dgs_status acquire_frame(dgs_ctx c, int64_t N, int64_t M, int64_t keys, int64_t tiles, int64_t pixels,
                         dgs_frame_s** out) {
    dgs_frame_s* f = nullptr;
    for (dgs_frame_s* x : c->frames)
        if (!x->live && (!f || x->cap_recs > f->cap_recs)) f = x;
    if (!f) {
        f = new dgs_frame_s();
        f->owner = c;
        c->frames.push_back(f);
    }
    hipError_t e = hipSuccess;
    if (!f->info && (e = hipMalloc((void**)&f->info, 16 * sizeof(uint32_t))) != hipSuccess) goto oom;
    if (M > f->cap_recs) {
        if ((e = grow(f->recs, M, c->stream)) != hipSuccess) goto oom;
        f->cap_recs = M;
    }
    if (N > f->cap_cells) {
        if ((e = grow(f->cell_v, N, c->stream)) != hipSuccess) goto oom;
        f->cap_cells = N;
    }
    if (keys > f->cap_vals) {
        if ((e = grow(f->vals, keys, c->stream)) != hipSuccess) goto oom;
        f->cap_vals = keys;
    }
    if (tiles > f->cap_tiles) {
        if ((e = grow(f->ranges, 2 * tiles, c->stream)) != hipSuccess) goto oom;
        if ((e = grow(f->order, 4 * tiles, c->stream)) != hipSuccess) goto oom;
        f->cap_tiles = tiles;
    }
    if (6 * pixels > f->cap_pix) {
        if ((e = grow(f->pix, 6 * pixels, c->stream)) != hipSuccess) goto oom;
        f->cap_pix = 6 * pixels;
    }
    *out = f;
    return DGS_OK;
oom:
    // drop the half-grown frame: its capacities no longer describe its buffers
    c->frames.erase(std::find(c->frames.begin(), c->frames.end(), f));
    free_frame(f);
    return fail(c, DGS_ERR_OOM, std::string("hipMalloc failed for a saved frame: ") + hipGetErrorString(e));
}

bool own_live_frame(dgs_ctx c, dgs_frame f) {
    return f && f->owner == c && f->live && std::find(c->frames.begin(), c->frames.end(), f) != c->frames.end();
}

// Copies the render's key total and statistics counters into a saved frame.
__global__ void k_frame_info(const uint32_t* misc, const unsigned long long* counters, uint32_t* info) {
    const int i = threadIdx.x;
    if (i == 0) info[2] = misc[0];
    if (i < 5) reinterpret_cast<unsigned long long*>(info + 4)[i] = counters[i];
}

}  // namespace

WorkspaceCaps dgs_internal_plan(const WorkspaceCaps& cur, const WorkspaceCaps& want) {
    WorkspaceCaps c = cur;
    if (want.prims > cur.prims) c.prims = want.prims + want.prims / 4;
    if (want.gauss > cur.gauss) c.gauss = want.gauss + want.gauss / 4;
    if (want.keys > cur.keys) c.keys = want.keys;
    if (want.tiles > cur.tiles) c.tiles = want.tiles;
    return c;
}

int64_t dgs_internal_bytes(const WorkspaceCaps& c) {
    int64_t b = 0;
    if (c.prims > 0)
        b += c.prims * (3 * 4 + 8 + 4 + 4 * 4) + (int64_t)(scan_status_words(c.prims) + sort_status_words(c.prims)) * 8;
    if (c.gauss > 0) b += c.gauss * ((int64_t)sizeof(GRec) + 8);
    if (c.keys > 0) b += c.keys * (2 * 8 + 2 * 4) + (int64_t)sort_status_words(c.keys) * 8;
    if (c.tiles > 0) b += c.tiles * (2 + 4) * 4;
    return b;
}

WorkspaceCaps dgs_internal_caps(dgs_ctx c) { return WorkspaceCaps{c->cap_prims, c->cap_gauss, c->cap_keys, c->cap_tiles}; }

void dgs_internal_release(dgs_ctx c) {
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    void** bufs[] = {(void**)&c->p_depth, (void**)&c->p_ntiles, (void**)&c->p_offsets, (void**)&c->p_rect,
                     (void**)&c->cell_v, (void**)&c->recs, (void**)&c->grect, (void**)&c->keys0,
                     (void**)&c->keys1, (void**)&c->vals0, (void**)&c->vals1, (void**)&c->ranges,
                     (void**)&c->tile_order, (void**)&c->scan_status, (void**)&c->sort_status,
                     (void**)&c->pk0, (void**)&c->pk1, (void**)&c->pv0, (void**)&c->pv1, (void**)&c->psort_status};
    for (void** p : bufs) {
        if (*p) hipFree(*p);
        *p = nullptr;
    }
    c->cap_prims = c->cap_gauss = c->cap_keys = c->cap_tiles = 0;
    c->scan_status_cap = c->sort_status_cap = 0;
    c->last_mode = -1;
    c->cur_ranges = nullptr;
    c->generation++;
}

dgs_status dgs_internal_frame(dgs_ctx c, const dgs_camera* cam, const dgs_render_opts* opts, const dgs_image* out,
                              FrameK* f, int* mode) {
    dgs_status st;
    if ((st = make_cam(c, cam, f->k)) != DGS_OK) return st;
    if ((st = make_opts(c, opts, f->o, *mode)) != DGS_OK) return st;
    if (!out || !out->color) return fail(c, DGS_ERR_INVALID_ARG, "output color buffer is NULL");
    f->color = out->color;
    f->D = out->weight_sum;
    f->T = out->final_T;
    f->last = out->last;
    f->sv_color = f->sv_D = f->sv_T = nullptr;
    f->sv_last = nullptr;
    return DGS_OK;
}

dgs_status dgs_internal_check_scene(dgs_ctx c, const dgs_scene* s, int mode) { return check_scene(c, s, mode); }

dgs_status dgs_internal_prepare(dgs_ctx c, const dgs_scene* s, int mode, int width, int height, int64_t keys) {
    const int64_t M = scene_gaussians(s);
    const int64_t P = mode != DGS_MODE_ALPHA ? s->num_cells : M;
    const int64_t tiles = (int64_t)((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
    hipSetDevice(c->device);
    return ensure(c, P, M, keys, tiles);
}

int64_t dgs_internal_default_keys(int64_t prims) { return prims * 8 > (1 << 20) ? prims * 8 : (1 << 20); }

extern "C" {

void dgs_default_opts(dgs_render_opts* o) {
    if (!o) return;
    o->mode = DGS_MODE_DUPLEX;
    o->flags = 0;
    o->eps_T = 1e-4f;
    o->alpha_min = 1.0f / 255.0f;
    o->alpha_max = 0.99f;
    o->cov2d_dilation = 0.3f;
    o->proxy_kappa = 1.0f;
    o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
    o->lcwsr_tau = 0.0f;
}

dgs_status dgs_create(int device, void* hip_stream, dgs_ctx* out) {
    if (!out) return DGS_ERR_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DGS_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return DGS_ERR_DEVICE;
    if (dgs_internal_noalloc_init(device) != hipSuccess) return DGS_ERR_DEVICE;
    dgs_ctx c = new dgs_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipMalloc((void**)&c->hist, 8 * 256 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void**)&c->misc, 16 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc((void**)&c->dev_err, sizeof(int)) != hipSuccess ||
        hipMalloc((void**)&c->counters, 5 * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&c->frame, sizeof(FrameK)) != hipSuccess ||
        hipHostMalloc((void**)&c->load_host, 2 * sizeof(uint64_t), hipHostMallocMapped) != hipSuccess) {
        dgs_destroy(c);
        return DGS_ERR_OOM;
    }
    c->load_host[0] = c->load_host[1] = 0;
    if (hipHostGetDevicePointer((void**)&c->load_dev, c->load_host, 0) != hipSuccess) {
        dgs_destroy(c);
        return DGS_ERR_DEVICE;
    }
    // the frame's second stream is created by the first frame that uses it
    // (ensure_aux), so contexts that never overlap inside a frame hold one
    // stream only
    hipMemsetAsync(c->misc, 0, 16 * sizeof(uint32_t), c->stream);
    hipMemsetAsync(c->dev_err, 0, sizeof(int), c->stream);
    hipMemsetAsync(c->counters, 0, 5 * sizeof(unsigned long long), c->stream);
    hipStreamSynchronize(c->stream);
    *out = c;
    return DGS_OK;
}

dgs_status dgs_destroy(dgs_ctx c) {
    if (!c) return DGS_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    if (c->aux) {
        hipStreamSynchronize(c->aux);
        hipStreamDestroy(c->aux);
    }
    if (c->ev_fork) hipEventDestroy(c->ev_fork);
    if (c->ev_join) hipEventDestroy(c->ev_join);
    for (auto& a : c->events)
        for (auto& e : a) hipEventDestroy(e);
    for (dgs_frame_s* f : c->frames) free_frame(f);
    c->frames.clear();
    void* ptrs[] = {c->p_depth, c->p_ntiles, c->p_offsets, c->p_rect, c->cell_v, c->recs, c->grect,
                    c->keys0, c->keys1, c->vals0, c->vals1, c->ranges, c->tile_order, c->scan_status, c->sort_status, c->g2d, c->gv, c->dec,
                    c->loss_coef, c->loss_part,
                    c->pk0, c->pk1, c->pv0, c->pv1, c->psort_status,
                    c->hist, c->misc, c->dev_err, c->counters, c->frame};
    for (void* p : ptrs)
        if (p) hipFree(p);
    if (c->load_host) hipHostFree(c->load_host);
    delete c;
    return DGS_OK;
}

dgs_status dgs_set_list_order(dgs_ctx c, int32_t order) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (order != DGS_LIST_ORDER_AUTO && order != DGS_LIST_ORDER_PER_TILE && order != DGS_LIST_ORDER_GLOBAL)
        return fail(c, DGS_ERR_INVALID_ARG, "list order must be DGS_LIST_ORDER_AUTO, _PER_TILE or _GLOBAL");
    c->list_order = order;
    return DGS_OK;
}

dgs_status dgs_set_overlap(dgs_ctx c, int32_t enable) {
    if (!c) return DGS_ERR_INVALID_ARG;
    c->two_streams = enable != 0;
    return DGS_OK;
}

dgs_status dgs_set_stream(dgs_ctx c, void* hip_stream) {
    if (!c) return DGS_ERR_INVALID_ARG;
    c->stream = (hipStream_t)hip_stream;
    return DGS_OK;
}

dgs_status dgs_reserve(dgs_ctx c, int64_t max_keys, int64_t max_prims, int64_t max_tiles) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (max_keys < 0 || max_prims < 0 || max_tiles < 0) return fail(c, DGS_ERR_INVALID_ARG, "negative size");
    hipSetDevice(c->device);
    return ensure(c, max_prims, max_prims, max_keys, max_tiles);
}

dgs_status dgs_render(dgs_ctx c, const dgs_scene* s, const dgs_camera* cam, const dgs_render_opts* opts,
                      const dgs_image* out, dgs_frame* saved) {
    if (!saved) return dgs_internal_render(c, s, cam, opts, out, true);
    if (!c) return DGS_ERR_INVALID_ARG;
    *saved = nullptr;
    CamK k;
    OptK o;
    int mode = 0;
    dgs_status st;
    if ((st = make_cam(c, cam, k)) != DGS_OK) return st;
    if ((st = make_opts(c, opts, o, mode)) != DGS_OK) return st;
    if (mode != DGS_MODE_DUPLEX) return fail(c, DGS_ERR_UNSUPPORTED, "only DGS_MODE_DUPLEX frames can be saved");
    if ((st = check_scene(c, s, mode)) != DGS_OK) return st;
    hipSetDevice(c->device);
    const int64_t N = s->num_cells, M = scene_gaussians(s);
    const int64_t tiles = (int64_t)k.TX * k.TY, pixels = (int64_t)k.W * k.H;
    const int64_t keys = c->cap_keys ? c->cap_keys : dgs_internal_default_keys(N);
    dgs_frame_s* f = nullptr;
    if ((st = acquire_frame(c, N, M, keys, tiles, pixels, &f)) != DGS_OK) return st;
    st = dgs_internal_render(c, s, cam, opts, out, true, nullptr, f);
    if (st != DGS_OK) return st;
    f->live = true;
    f->k = k;
    f->o = o;
    f->N = (int)N;
    f->K = s->gaussians_per_cell;
    f->offs = s->cell_offsets;
    f->M = M;
    f->tiles = (int)tiles;
    *saved = f;
    return DGS_OK;
}

dgs_status dgs_render_neural(dgs_ctx c, const dgs_neural_scene* ns, const dgs_decoder* dec, const dgs_camera* cam,
                             const dgs_render_opts* opts, const dgs_image* out) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (!ns || !dec) return fail(c, DGS_ERR_INVALID_ARG, "neural scene or decoder is NULL");
    if (ns->num_cells < 0) return fail(c, DGS_ERR_INVALID_ARG, "num_cells < 0");
    if (ns->gaussians_per_cell < 1 || ns->gaussians_per_cell > kMaxK)
        return fail(c, DGS_ERR_INVALID_ARG, "gaussians_per_cell must be in 1..32");
    if (dec->feature_dim < 1 || dec->feature_dim > kMaxFeature || dec->hidden_dim < 1 ||
        dec->hidden_dim > kMaxHidden)
        return fail(c, DGS_ERR_INVALID_ARG, "feature_dim and hidden_dim must be in 1..64");
    if (ns->num_cells > 0 && (!ns->features || !ns->offsets || !dec->weights))
        return fail(c, DGS_ERR_INVALID_ARG, "features, offsets and decoder weights must not be NULL");
    const int64_t M = (int64_t)ns->num_cells * ns->gaussians_per_cell;
    if (M > (int64_t)(1 << 30)) return fail(c, DGS_ERR_INVALID_ARG, "too many Gaussians");
    hipSetDevice(c->device);
    if (14 * M > c->cap_dec) {
        hipError_t e = grow(c->dec, 14 * M, c->stream);
        if (e != hipSuccess) {
            c->cap_dec = 0;
            return fail(c, DGS_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        }
        c->cap_dec = 14 * M;
    }
    dgs_scene s;
    s.num_cells = ns->num_cells;
    s.gaussians_per_cell = ns->gaussians_per_cell;
    s.cell_pos = ns->cell_pos;
    s.cell_scale = ns->cell_scale;
    s.cell_rot = ns->cell_rot;
    s.cell_v_sh = ns->cell_v_sh;
    s.v_sh_degree = ns->v_sh_degree;
    s.means = c->dec;
    s.scales = c->dec + 3 * M;
    s.rots = c->dec + 6 * M;
    s.opacities = c->dec + 10 * M;
    s.sh = c->dec + 11 * M;
    s.sh_degree = -1;
    s.cell_offsets = nullptr;
    s.num_gaussians = 0;
    const NeuralSrc nn{ns, dec};
    dgs_status st = dgs_internal_render(c, &s, cam, opts, out, true, &nn);
    if (st == DGS_OK) c->dec_gauss = M;
    return st;
}

dgs_status dgs_read_decoded(dgs_ctx c, float* means, float* scales, float* rots, float* opacities, float* colors) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (c->last_mode < 0 || !c->last_neural) return fail(c, DGS_ERR_INVALID_ARG, "the last render was not neural");
    hipSetDevice(c->device);
    const int64_t M = c->dec_gauss;
    float* dst[5] = {means, scales, rots, opacities, colors};
    const int64_t off[5] = {0, 3 * M, 6 * M, 10 * M, 11 * M}, len[5] = {3 * M, 3 * M, 4 * M, M, 3 * M};
    for (int i = 0; i < 5; i++)
        if (dst[i] && len[i] > 0)
            hipMemcpyAsync(dst[i], c->dec + off[i], sizeof(float) * (size_t)len[i], hipMemcpyDeviceToDevice,
                           c->stream);
    return launched(c);
}

}  // extern "C"

// Per-cell tile lists (Duplex, LC-WSR) are put in depth order per tile
// (launch_tile_depth_sort) when the context's last cell frame had at most 8
// keys per cell, at most 1024 keys per tile on
// average, and at most a twentieth of its keys in runs of more than 4096
// entries (which the per-tile sort handles by chunked merges in global
// memory over several rounds); before any cell frame, when the key buffer
// holds at most 256 keys per tile.  The per-tile sort's cost grows with the keys and their
// run lengths, the depth sort's with the cells only.  Per-Gaussian lists
// always take the depth sort of the primitives.
constexpr uint64_t kPerTileOrderKeysPerCell = 8;
constexpr int64_t kPerTileOrderMaxMean = 1024;      // keys per tile
constexpr uint64_t kPerTileOrderLongShare = 20;     // at most 1 / this of the keys in long runs
constexpr int64_t kPerTileOrderCapacity = 256;      // keys per tile, before any cell frame

static bool per_tile_order(dgs_ctx c, int64_t tiles, bool cells) {
    if (c->list_order == DGS_LIST_ORDER_PER_TILE) return true;
    if (c->list_order == DGS_LIST_ORDER_GLOBAL) return false;
    if (!cells) return false;
    const uint64_t load = __atomic_load_n(c->load_host, __ATOMIC_RELAXED);
    const uint64_t lng = __atomic_load_n(c->load_host + 1, __ATOMIC_RELAXED);
    const uint64_t lt = load >> 32, lk = load & 0xffffffffull, lp = lng >> 32, ll = lng & 0xffffffffull;
    if (lt)
        return lk <= kPerTileOrderKeysPerCell * lp && lk <= (uint64_t)kPerTileOrderMaxMean * lt &&
               kPerTileOrderLongShare * ll <= lk;
    return c->cap_keys <= kPerTileOrderCapacity * tiles;
}

// The context's second stream and its fork/join events, created on first
// use.  Not while the context's stream is being captured into a graph (a
// stream cannot be created inside a capture): such a frame runs on one
// stream.  False when the second stream is not available.
static bool ensure_aux(dgs_ctx c) {
    if (c->aux) return true;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return false;
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
        c->aux = nullptr;
        return false;
    }
    if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        if (c->ev_fork) hipEventDestroy(c->ev_fork);
        if (c->ev_join) hipEventDestroy(c->ev_join);
        hipStreamDestroy(c->aux);
        c->aux = nullptr;
        c->ev_fork = c->ev_join = nullptr;
        return false;
    }
    return true;
}

// The frame pipeline.  With write_frame the frame's camera and options are
// written to the context's device FrameK by the first kernel; without it the
// caller has put them there (a captured graph replayed for a new camera).
dgs_status dgs_internal_render(dgs_ctx c, const dgs_scene* s, const dgs_camera* cam, const dgs_render_opts* opts,
                               const dgs_image* out, bool write_frame, const NeuralSrc* nn, dgs_frame_s* save) {
    if (!c) return DGS_ERR_INVALID_ARG;
    CamK k;
    OptK o;
    int mode = 0;
    dgs_status st;
    if ((st = make_cam(c, cam, k)) != DGS_OK) return st;
    if ((st = make_opts(c, opts, o, mode)) != DGS_OK) return st;
    if ((st = check_scene(c, s, mode, nn != nullptr)) != DGS_OK) return st;
    if (!out || !out->color) return fail(c, DGS_ERR_INVALID_ARG, "output color buffer is NULL");
    hipSetDevice(c->device);
    const int N = s->num_cells, K = s->gaussians_per_cell;
    const int M = (int)scene_gaussians(s);
    const int tiles = k.TX * k.TY;
    const bool cells = mode != DGS_MODE_ALPHA;
    const int P = cells ? N : M;
    int64_t want_keys = c->cap_keys;
    if (want_keys == 0) want_keys = dgs_internal_default_keys(P);
    if ((st = ensure(c, P, M, want_keys, tiles)) != DGS_OK) return st;
    const uint32_t cap = (uint32_t)c->cap_keys;
    hipStream_t q = c->stream;
    const bool overlap = cells && !c->timing && c->two_streams && ensure_aux(c);
    // the lists' depth order: a depth sort of the primitives (ties by id)
    // before the key emission, or, when the tile lists are short, a sort of
    // each tile's run after the tile sort (the same order); with the second
    // stream, the work queue is then built there beside the per-tile sort
    const bool per_tile = per_tile_order(c, tiles, cells);
    // buffers the backward replays: a saved frame's own, else the context's
    float* cell_v = save ? save->cell_v : c->cell_v;
    GRec* recs = save ? save->recs : c->recs;
    uint32_t* ranges = save ? save->ranges : c->ranges;
    uint32_t* torder = save ? save->order : c->tile_order;
    uint32_t* queue = save ? save->info : c->misc + 11;

    StageMarks sm(c);
    {
        // per-frame zeroing: digit histograms, scan/sort tickets and the
        // compositor queue (misc[1..12]), tile ranges, statistics counters
        ClearList cl;
        cl.add(c->hist, 8 * 256);
        cl.add(c->misc + 1, 12);
        cl.add(ranges, 2 * (size_t)tiles);
        if (o.stats || save) cl.add((uint32_t*)c->counters, 10);
        cl.bump = c->misc + 13;
        FrameK f{k, o, out->color, out->weight_sum, out->final_T, out->last, nullptr, nullptr, nullptr, nullptr};
        if (save) {
            const size_t HW = (size_t)k.W * k.H;
            f.sv_color = save->pix;
            f.sv_D = save->pix + 3 * HW;
            f.sv_T = save->pix + 4 * HW;
            f.sv_last = reinterpret_cast<int32_t*>(save->pix + 5 * HW);
        }
        launch_clear(q, cl, write_frame ? &f : nullptr, c->frame);
    }
    sm.mark(0);
    // Duplex / LC-WSR: the cell sort needs only the cell preprocess, so the
    // (decode and) projection of the members runs on the second stream
    // meanwhile; with stage timing on, everything stays on one stream
    if (cells) {
        launch_cell_preprocess(q, N, s->cell_pos, s->cell_scale, s->cell_rot, s->cell_v_sh, s->v_sh_degree,
                               s->cell_offsets, M, K, c->frame, c->p_depth, c->p_rect, c->p_ntiles, cell_v,
                               c->dev_err);
        hipStream_t pq = q;
        if (overlap) {
            hipEventRecord(c->ev_fork, q);
            hipStreamWaitEvent(c->aux, c->ev_fork, 0);
            pq = c->aux;
        }
        if (nn) launch_decode(pq, decode_args(c, *nn, c->p_ntiles));
        sm.mark(1);
        // fixed layout: members of culled cells are skipped (the cell of
        // Gaussian g is g / K); ragged cells: every Gaussian is projected
        launch_gauss_project(pq, M, K, s->means, s->scales, s->rots, s->opacities, s->sh, s->sh_degree, c->frame,
                             s->cell_offsets ? nullptr : c->p_ntiles, recs, c->grect, nullptr, nullptr, overlap);
        if (overlap) hipEventRecord(c->ev_join, c->aux);
    } else {
        if (nn) launch_decode(q, decode_args(c, *nn, nullptr));
        sm.mark(1);
        launch_gauss_project(q, M, K, s->means, s->scales, s->rots, s->opacities, s->sh, s->sh_degree, c->frame,
                             nullptr, recs, c->grect, c->p_depth, c->p_ntiles);
    }
    sm.mark(2);
    const uint64_t* prect = cells ? c->p_rect : c->grect;
    const uint32_t* order = nullptr;  // null: keys emitted in primitive-id order
    if (!per_tile) {
        launch_prim_keys(q, P, c->p_ntiles, c->p_depth, c->pk0, c->pv0, c->hist);
        const SortScratch ps{c->hist, c->psort_status, c->misc + 2};
        const bool pin1 = launch_radix_sort32(q, c->pk0, c->pv0, c->pk1, c->pv1, (uint32_t)P, ps, c->misc + 13, 1,
                                              c->dev_err);
        order = pin1 ? c->pv1 : c->pv0;
    }
    sm.mark(3);
    launch_exclusive_scan(q, c->p_ntiles, c->p_offsets, P, c->misc + 0, c->scan_status, c->misc + 13, c->misc + 1,
                          c->dev_err, order);
    const int tbits = tile_bits(tiles);
    launch_emit_keys(q, P, order, c->p_ntiles, c->p_offsets, prect, c->p_depth, k.TX, cap, c->keys0, c->vals0,
                     c->hist + 4 * 256, sort_passes(tbits), c->dev_err);
    sm.mark(4);
    // stable sort on the tile bits
    const SortScratch ss{c->hist + 4 * 256, c->sort_status, c->misc + 6};
    const bool in1 = launch_radix_sort(q, c->keys0, c->vals0, c->keys1, c->vals1, c->misc + 0, cap, tbits, ss,
                                       c->misc + 13, c->dev_err, true, 32, 5);
    uint64_t* skeys = in1 ? c->keys1 : c->keys0;
    uint32_t* svals = in1 ? c->vals1 : c->vals0;
    sm.mark(5);
    launch_tile_ranges(q, skeys, c->misc + 0, cap, ranges, svals, save && !per_tile ? save->vals : nullptr,
                       cells ? c->load_dev : nullptr, (uint32_t)tiles);
    sm.mark(6);
    // per tile: the same launch also builds the work queue
    if (per_tile)
        launch_tile_depth_sort(q, ranges, tiles, skeys, svals, in1 ? c->keys0 : c->keys1,
                               save ? save->vals : nullptr, cells ? kSplitLenCells : kSplitLenGauss, torder, queue,
                               cells ? c->load_dev + 1 : nullptr, (uint32_t)P);
    sm.mark(7);
    CompositeArgs a;
    a.ranges = ranges;
    a.vals = svals;
    a.recs = recs;
    a.cell_v = cell_v;
    a.offs = cells ? s->cell_offsets : nullptr;
    a.K = K;
    a.fr = c->frame;
    a.k = k;  // host copy: grid sizes only
    a.o = o;
    a.color = out->color;
    a.D = out->weight_sum;
    a.T = out->final_T;
    a.last = out->last;
    a.counters = o.stats ? c->counters : nullptr;
    a.order = torder;
    a.queue = queue;
    a.save = save != nullptr;
    if (!per_tile)
        launch_tile_order(q, ranges, tiles, cells ? kSplitLenCells : kSplitLenGauss, torder, queue,
                          cells ? c->load_dev + 1 : nullptr, (uint32_t)P);
    if (overlap) hipStreamWaitEvent(q, c->ev_join, 0);  // the projected members
    sm.mark(8);
    if (mode == DGS_MODE_DUPLEX)
        launch_composite_duplex(q, a);
    else if (mode == DGS_MODE_LCWSR)
        launch_composite_lcwsr(q, a);
    else
        launch_composite_alpha(q, a);
    sm.mark(9);
    if (save) hipLaunchKernelGGL(k_frame_info, dim3(1), dim3(64), 0, q, c->misc, c->counters, save->info);
    c->cur_ranges = ranges;
    c->last_mode = mode;
    c->last_neural = nn != nullptr;
    c->last_passes = (P > 0 && !per_tile ? sort_passes(32) : 0) + sort_passes(tbits);
    c->last_prims = P;
    c->last_gauss = M;
    c->last_tiles = tiles;
    c->last_in_1 = in1;
    return launched(c);
}

extern "C" {

dgs_status dgs_render_backward(dgs_ctx c, const dgs_scene* s, const dgs_camera* cam, const dgs_render_opts* opts,
                               dgs_frame f, const float* grad_color, const float* grad_weight_sum,
                               const dgs_grads* gr) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (!own_live_frame(c, f)) return fail(c, DGS_ERR_INVALID_ARG, "not a live saved frame of this context");
    dgs_status st;
    if (cam) {
        CamK k;
        memset(&k, 0, sizeof k);
        if ((st = make_cam(c, cam, k)) != DGS_OK) return st;
        if (memcmp(&k, &f->k, sizeof k) != 0) return fail(c, DGS_ERR_INVALID_ARG, "camera differs from the saved frame's");
    }
    if (opts) {
        OptK o;
        int mode = 0;
        memset(&o, 0, sizeof o);
        if ((st = make_opts(c, opts, o, mode)) != DGS_OK) return st;
        if (mode != DGS_MODE_DUPLEX) return fail(c, DGS_ERR_UNSUPPORTED, "backward is implemented for DGS_MODE_DUPLEX");
        o.stats = f->o.stats;  // counting does not change the frame
        if (memcmp(&o, &f->o, sizeof o) != 0)
            return fail(c, DGS_ERR_INVALID_ARG, "render options differ from the saved frame's");
    }
    if ((st = check_scene(c, s, DGS_MODE_DUPLEX)) != DGS_OK) return st;
    if (!grad_color || !gr) return fail(c, DGS_ERR_INVALID_ARG, "grad_color and grads must not be NULL");
    if (!gr->d_means || !gr->d_scales || !gr->d_rots || !gr->d_opacities || !gr->d_sh || !gr->d_cell_v_sh ||
        !gr->d_cell_pos)
        return fail(c, DGS_ERR_INVALID_ARG, "gradient buffers must not be NULL (only d_mean2d is optional)");
    const int N = s->num_cells, K = s->gaussians_per_cell, M = (int)scene_gaussians(s);
    if (N != f->N || K != f->K || M != f->M || s->cell_offsets != f->offs)
        return fail(c, DGS_ERR_INVALID_ARG, "scene sizes or layout differ from the saved frame's");
    if (M == 0) return DGS_OK;
    hipSetDevice(c->device);
    hipError_t e = hipSuccess;
    if (kG2dRow * (int64_t)M > c->cap_g2d) {
        if ((e = grow(c->g2d, kG2dRow * (int64_t)M, c->stream)) != hipSuccess) goto oom;
        c->cap_g2d = kG2dRow * (int64_t)M;
    }
    if (N > c->cap_gv) {
        if ((e = grow(c->gv, (int64_t)N, c->stream)) != hipSuccess) goto oom;
        c->cap_gv = N;
    }
    {
        hipStream_t q = c->stream;
        const size_t HW = (size_t)f->k.W * f->k.H;
        float* color = f->pix;
        float* D = f->pix + 3 * HW;
        float* T = f->pix + 4 * HW;
        int32_t* last = reinterpret_cast<int32_t*>(f->pix + 5 * HW);
        launch_fill_u32(q, (uint32_t*)c->g2d, 0u, kG2dRow * (size_t)M);
        launch_fill_u32(q, (uint32_t*)c->gv, 0u, (size_t)N);
        // the forward's work queue (same ranges, same split) is in the
        // frame with its item count: rewind its head only
        launch_fill_u32(q, f->info, 0u, 1);
        launch_set_frame(q, FrameK{f->k, f->o, color, D, T, last, nullptr, nullptr, nullptr, nullptr}, c->frame);
        BwdArgs a;
        a.ranges = f->ranges;
        a.vals = f->vals;
        a.recs = f->recs;
        a.cell_v = f->cell_v;
        a.offs = f->offs;
        a.K = K;
        a.M = M;
        a.fr = c->frame;
        a.k = f->k;
        a.o = f->o;
        a.color = color;
        a.D = D;
        a.T = T;
        a.last = last;
        a.grad_color = grad_color;
        a.grad_D = grad_weight_sum;
        a.g2d = c->g2d;
        a.gv = c->gv;
        a.order = f->order;
        a.queue = f->info;
        launch_composite_bwd(q, a);
        ProjBwdArgs b;
        b.N = N;
        b.means = s->means;
        b.scales = s->scales;
        b.rots = s->rots;
        b.sh = s->sh;
        b.sh_degree = s->sh_degree;
        b.cell_pos = s->cell_pos;
        b.cell_v_sh = s->cell_v_sh;
        b.v_sh_degree = s->v_sh_degree;
        b.d_means = gr->d_means;
        b.d_scales = gr->d_scales;
        b.d_rots = gr->d_rots;
        b.d_opac = gr->d_opacities;
        b.d_sh = gr->d_sh;
        b.d_cell_v_sh = gr->d_cell_v_sh;
        b.d_cell_pos = gr->d_cell_pos;
        b.overwrite = gr->overwrite != 0;
        b.d_mean2d = gr->d_mean2d;
        launch_project_bwd(q, a, b);
    }
    return launched(c);
oom:
    return fail(c, DGS_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
}

dgs_status dgs_frame_release(dgs_ctx c, dgs_frame f) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (!own_live_frame(c, f)) return fail(c, DGS_ERR_INVALID_ARG, "not a live saved frame of this context");
    f->live = false;
    return DGS_OK;
}

dgs_status dgs_frame_stats(dgs_ctx c, dgs_frame f, dgs_stats* out) {
    if (!c || !out) return DGS_ERR_INVALID_ARG;
    if (!own_live_frame(c, f)) return fail(c, DGS_ERR_INVALID_ARG, "not a live saved frame of this context");
    hipSetDevice(c->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, DGS_ERR_DEVICE, "stream synchronize failed");
    uint32_t info[16];
    if (hipMemcpy(info, f->info, sizeof info, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, DGS_ERR_DEVICE, "frame counters readback failed");
    unsigned long long cnt[5];
    memcpy(cnt, info + 4, sizeof cnt);
    memset(out, 0, sizeof *out);
    out->num_keys = info[2];
    out->key_capacity = f->cap_vals;
    out->n_val = (int64_t)cnt[0];
    out->n_rendered = (int64_t)cnt[1];
    out->n_box = (int64_t)cnt[2];
    out->n_cell_hits = (int64_t)cnt[3];
    out->n_cell_pixels = (int64_t)cnt[4];
    return DGS_OK;
}

dgs_status dgs_sync(dgs_ctx c) {
    if (!c) return DGS_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, DGS_ERR_DEVICE, "stream synchronize failed");
    int e = 0;
    if (hipMemcpy(&e, c->dev_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, DGS_ERR_DEVICE, "error flag readback failed");
    if (e) {
        // cleared in stream order, before the next frame can set a flag
        launch_fill_u32(c->stream, reinterpret_cast<uint32_t*>(c->dev_err), 0u, 1);
        if (e & (1 << kErrTimeout)) return fail(c, DGS_ERR_TIMEOUT, timeout_message(e));
        if (e & (1 << kErrInvalid))
            return fail(c, DGS_ERR_INVALID_ARG, "malformed cell_offsets (those cells were culled)");
        if (e & (1 << kErrCapacity)) return fail(c, DGS_ERR_CAPACITY, "key capacity exceeded; reserve more keys");
        return fail(c, DGS_ERR_DEVICE, "device error flag set");
    }
    return DGS_OK;
}

dgs_status dgs_get_stats(dgs_ctx c, dgs_stats* out) {
    if (!c || !out) return DGS_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, DGS_ERR_DEVICE, "stream synchronize failed");
    uint32_t total = 0;
    unsigned long long cnt[5] = {0, 0, 0, 0, 0};
    int e = 0;
    hipMemcpy(&total, c->misc, sizeof(uint32_t), hipMemcpyDeviceToHost);
    hipMemcpy(cnt, c->counters, sizeof(cnt), hipMemcpyDeviceToHost);
    hipMemcpy(&e, c->dev_err, sizeof(int), hipMemcpyDeviceToHost);
    out->num_keys = total;
    out->key_capacity = c->cap_keys;
    out->n_val = (int64_t)cnt[0];
    out->n_rendered = (int64_t)cnt[1];
    out->n_box = (int64_t)cnt[2];
    out->n_cell_hits = (int64_t)cnt[3];
    out->n_cell_pixels = (int64_t)cnt[4];
    out->device_error = (e & (1 << kErrTimeout))    ? DGS_ERR_TIMEOUT
                        : (e & (1 << kErrInvalid))  ? DGS_ERR_INVALID_ARG
                        : (e & (1 << kErrCapacity)) ? DGS_ERR_CAPACITY
                                                    : 0;
    out->sort_passes = c->last_passes;
    return DGS_OK;
}

const char* dgs_last_error(dgs_ctx c) { return c ? c->err.c_str() : "invalid context"; }

dgs_status dgs_read_lists(dgs_ctx c, uint64_t* keys, uint32_t* values, uint32_t* ranges) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (c->last_mode < 0) return fail(c, DGS_ERR_INVALID_ARG, "no frame rendered yet");
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    uint32_t total = 0;
    hipMemcpy(&total, c->misc, sizeof(uint32_t), hipMemcpyDeviceToHost);
    if ((int64_t)total > c->cap_keys) total = (uint32_t)c->cap_keys;
    const uint64_t* sk = c->last_in_1 ? c->keys1 : c->keys0;
    const uint32_t* sv = c->last_in_1 ? c->vals1 : c->vals0;
    if (keys && total) hipMemcpyAsync(keys, sk, total * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream);
    if (values && total) hipMemcpyAsync(values, sv, total * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream);
    if (ranges && c->cur_ranges)
        hipMemcpyAsync(ranges, c->cur_ranges, 2 * c->last_tiles * sizeof(uint32_t), hipMemcpyDeviceToDevice,
                       c->stream);
    return launched(c);
}

dgs_status dgs_read_prims(dgs_ctx c, int32_t* rect, uint32_t* depth_bits, uint32_t* ntiles) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (c->last_mode < 0) return fail(c, DGS_ERR_INVALID_ARG, "no frame rendered yet");
    hipSetDevice(c->device);
    const int64_t P = c->last_prims;
    if (P == 0) return DGS_OK;
    const uint64_t* pr = c->last_mode != DGS_MODE_ALPHA ? c->p_rect : c->grect;
    if (rect) hipLaunchKernelGGL(k_unpack_rects, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, c->stream, pr, P, rect);
    if (depth_bits) hipMemcpyAsync(depth_bits, c->p_depth, P * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream);
    if (ntiles) hipMemcpyAsync(ntiles, c->p_ntiles, P * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream);
    return launched(c);
}

dgs_status dgs_read_gauss_rects(dgs_ctx c, int32_t* rect) {
    if (!c || !rect) return DGS_ERR_INVALID_ARG;
    if (c->last_mode < 0) return fail(c, DGS_ERR_INVALID_ARG, "no frame rendered yet");
    hipSetDevice(c->device);
    const int64_t M = c->last_gauss;
    if (M == 0) return DGS_OK;
    hipLaunchKernelGGL(k_unpack_rects, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, c->stream, c->grect, M, rect);
    return launched(c);
}

dgs_status dgs_set_timing(dgs_ctx c, int32_t enable) {
    if (!c) return DGS_ERR_INVALID_ARG;
    c->timing = enable != 0;
    return DGS_OK;
}

dgs_status dgs_get_timing(dgs_ctx c, float* ms, int32_t n_stages, int32_t* frames) {
    if (!c || !ms || n_stages < 0 || n_stages > DGS_NUM_STAGES) return DGS_ERR_INVALID_ARG;
    hipSetDevice(c->device);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, DGS_ERR_DEVICE, "stream synchronize failed");
    for (int i = 0; i < n_stages; i++) ms[i] = 0.0f;
    for (size_t f = 0; f < c->events_used; f++) {
        auto& ev = c->events[f];
        for (int i = 0; i < n_stages; i++) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, ev[i], ev[i + 1]) == hipSuccess) ms[i] += t;
        }
    }
    if (frames) *frames = (int32_t)c->events_used;
    c->events_used = 0;
    return DGS_OK;
}

dgs_status dgs_sort_pairs(dgs_ctx c, uint64_t* keys, uint32_t* values, int64_t n, int32_t key_bits) {
    if (!c) return DGS_ERR_INVALID_ARG;
    if (n < 0 || key_bits < 1 || key_bits > 64) return fail(c, DGS_ERR_INVALID_ARG, "bad n or key_bits");
    if (n == 0) return DGS_OK;
    if (!keys || !values) return fail(c, DGS_ERR_INVALID_ARG, "NULL buffer");
    hipSetDevice(c->device);
    dgs_status st;
    if ((st = ensure(c, 0, 0, n, 0)) != DGS_OK) return st;
    c->last_mode = -1;  // the sort overwrites the last render's sorted lists (saved frames keep their own)
    ClearList cl;
    cl.add(c->hist, 8 * 256);
    cl.add(c->misc + 2, 8);
    cl.bump = c->misc + 13;
    launch_clear(c->stream, cl);
    launch_fill_u32(c->stream, c->misc + 10, (uint32_t)n, 1);
    SortScratch ss{c->hist, c->sort_status, c->misc + 2};
    const bool in1 = launch_radix_sort(c->stream, keys, values, c->keys1, c->vals1, c->misc + 10, (uint32_t)n,
                                       key_bits, ss, c->misc + 13, c->dev_err);
    if (in1) {
        hipMemcpyAsync(keys, c->keys1, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->stream);
        hipMemcpyAsync(values, c->vals1, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->stream);
    }
    return launched(c);
}

}  // extern "C"
