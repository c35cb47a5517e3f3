"""ctypes binding of include/duplexgs.h (argument marshalling only).

The functions keep the C names.  Loading fails loudly when the HIP library
has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libduplexgs.so")

DGS_OK = 0
DGS_ERR_INVALID_ARG = 1
DGS_ERR_OOM = 2
DGS_ERR_CAPACITY = 3
DGS_ERR_DEVICE = 4
DGS_ERR_UNSUPPORTED = 5
DGS_ERR_TIMEOUT = 6
STATUS_NAMES = {0: "DGS_OK", 1: "DGS_ERR_INVALID_ARG", 2: "DGS_ERR_OOM", 3: "DGS_ERR_CAPACITY",
                4: "DGS_ERR_DEVICE", 5: "DGS_ERR_UNSUPPORTED", 6: "DGS_ERR_TIMEOUT"}

DGS_MODE_DUPLEX = 0
DGS_MODE_ALPHA = 1
DGS_MODE_LCWSR = 2
DGS_FLAG_V_ONE = 1
DGS_FLAG_NO_ET = 2
DGS_FLAG_STATS = 4


class dgs_scene(C.Structure):
    _fields_ = [("num_cells", C.c_int32), ("gaussians_per_cell", C.c_int32),
                ("cell_pos", C.c_void_p), ("cell_scale", C.c_void_p), ("cell_rot", C.c_void_p),
                ("cell_v_sh", C.c_void_p), ("v_sh_degree", C.c_int32),
                ("means", C.c_void_p), ("scales", C.c_void_p), ("rots", C.c_void_p),
                ("opacities", C.c_void_p), ("sh", C.c_void_p), ("sh_degree", C.c_int32),
                ("cell_offsets", C.c_void_p), ("num_gaussians", C.c_int32)]


class dgs_camera(C.Structure):
    _fields_ = [("viewmat", C.c_float * 16), ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float),
                ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32), ("z_near", C.c_float)]


class dgs_render_opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("flags", C.c_uint32), ("eps_T", C.c_float), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("cov2d_dilation", C.c_float), ("proxy_kappa", C.c_float),
                ("bg", C.c_float * 3), ("lcwsr_tau", C.c_float)]


class dgs_image(C.Structure):
    _fields_ = [("color", C.c_void_p), ("weight_sum", C.c_void_p), ("final_T", C.c_void_p), ("last", C.c_void_p)]


class dgs_grads(C.Structure):
    _fields_ = [("d_means", C.c_void_p), ("d_scales", C.c_void_p), ("d_rots", C.c_void_p),
                ("d_opacities", C.c_void_p), ("d_sh", C.c_void_p), ("d_cell_v_sh", C.c_void_p),
                ("d_cell_pos", C.c_void_p), ("d_mean2d", C.c_void_p), ("overwrite", C.c_int32)]


class dgs_stats(C.Structure):
    _fields_ = [("num_keys", C.c_int64), ("key_capacity", C.c_int64), ("n_val", C.c_int64),
                ("n_rendered", C.c_int64), ("n_box", C.c_int64), ("n_cell_hits", C.c_int64),
                ("device_error", C.c_int32), ("sort_passes", C.c_int32), ("n_cell_pixels", C.c_int64)]


class dgs_decoder(C.Structure):
    _fields_ = [("feature_dim", C.c_int32), ("hidden_dim", C.c_int32), ("weights", C.c_void_p)]


class dgs_neural_scene(C.Structure):
    _fields_ = [("num_cells", C.c_int32), ("gaussians_per_cell", C.c_int32),
                ("cell_pos", C.c_void_p), ("cell_scale", C.c_void_p), ("cell_rot", C.c_void_p),
                ("cell_v_sh", C.c_void_p), ("v_sh_degree", C.c_int32), ("features", C.c_void_p),
                ("offsets", C.c_void_p)]


class dgs_server_config(C.Structure):
    _fields_ = [("num_slots", C.c_int32), ("use_graphs", C.c_int32), ("memory_budget", C.c_int64)]


class dgs_sim_device(C.Structure):
    _fields_ = [("seconds_fixed", C.c_double), ("seconds_per_mpixel", C.c_double), ("keys_per_pixel", C.c_double)]


class dgs_request_info(C.Structure):
    _fields_ = [("state", C.c_int32), ("result", C.c_int32), ("slot", C.c_int32), ("attempts", C.c_int32),
                ("graph", C.c_int32), ("reserved", C.c_int32), ("num_keys", C.c_int64), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


class dgs_server_stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("submitted", "completed", "failed", "cancelled", "retries",
                                          "graph_captures", "graph_replays", "releases", "workspace_bytes",
                                          "peak_workspace_bytes", "queued", "running")]


DGS_REQ_QUEUED, DGS_REQ_RUNNING, DGS_REQ_DONE, DGS_REQ_FAILED, DGS_REQ_CANCELLED = range(5)

dgs_ctx = C.c_void_p
dgs_frame = C.c_void_p
dgs_server = C.c_void_p

# name -> (restype, argtypes)
_SIGS = {
    "dgs_default_opts": (None, [C.POINTER(dgs_render_opts)]),
    "dgs_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(dgs_ctx)]),
    "dgs_destroy": (C.c_int, [dgs_ctx]),
    "dgs_set_stream": (C.c_int, [dgs_ctx, C.c_void_p]),
    "dgs_reserve": (C.c_int, [dgs_ctx, C.c_int64, C.c_int64, C.c_int64]),
    "dgs_render": (C.c_int, [dgs_ctx, C.POINTER(dgs_scene), C.POINTER(dgs_camera), C.POINTER(dgs_render_opts),
                             C.POINTER(dgs_image), C.POINTER(dgs_frame)]),
    "dgs_render_backward": (C.c_int, [dgs_ctx, C.POINTER(dgs_scene), C.POINTER(dgs_camera),
                                      C.POINTER(dgs_render_opts), dgs_frame, C.c_void_p, C.c_void_p,
                                      C.POINTER(dgs_grads)]),
    "dgs_frame_release": (C.c_int, [dgs_ctx, dgs_frame]),
    "dgs_frame_stats": (C.c_int, [dgs_ctx, dgs_frame, C.POINTER(dgs_stats)]),
    "dgs_render_neural": (C.c_int, [dgs_ctx, C.POINTER(dgs_neural_scene), C.POINTER(dgs_decoder),
                                    C.POINTER(dgs_camera), C.POINTER(dgs_render_opts), C.POINTER(dgs_image)]),
    "dgs_read_decoded": (C.c_int, [dgs_ctx, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dgs_sync": (C.c_int, [dgs_ctx]),
    "dgs_get_stats": (C.c_int, [dgs_ctx, C.POINTER(dgs_stats)]),
    "dgs_last_error": (C.c_char_p, [dgs_ctx]),
    "dgs_read_lists": (C.c_int, [dgs_ctx, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dgs_read_prims": (C.c_int, [dgs_ctx, C.c_void_p, C.c_void_p, C.c_void_p]),
    "dgs_read_gauss_rects": (C.c_int, [dgs_ctx, C.c_void_p]),
    "dgs_sort_pairs": (C.c_int, [dgs_ctx, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "dgs_sort_pairs_noalloc": (C.c_int, [dgs_ctx, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32]),
    "dgs_set_list_order": (C.c_int, [dgs_ctx, C.c_int32]),
    "dgs_set_overlap": (C.c_int, [dgs_ctx, C.c_int32]),
    "dgs_loss_l1_ssim": (C.c_int, [dgs_ctx, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_float,
                                   C.c_void_p, C.c_void_p]),
    "dgs_set_timing": (C.c_int, [dgs_ctx, C.c_int32]),
    "dgs_get_timing": (C.c_int, [dgs_ctx, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_int32)]),
    "dgs_server_default_config": (None, [C.POINTER(dgs_server_config)]),
    "dgs_server_create": (C.c_int, [C.c_int, C.POINTER(dgs_server_config), C.POINTER(dgs_server)]),
    "dgs_server_create_simulated": (C.c_int, [C.POINTER(dgs_server_config), C.POINTER(dgs_sim_device),
                                              C.POINTER(dgs_server)]),
    "dgs_server_add_scene": (C.c_int, [dgs_server, C.POINTER(dgs_scene), C.POINTER(C.c_int32)]),
    "dgs_server_submit": (C.c_int, [dgs_server, C.c_int32, C.POINTER(dgs_camera), C.POINTER(dgs_render_opts),
                                    C.POINTER(dgs_image), C.POINTER(C.c_int64)]),
    "dgs_server_query": (C.c_int, [dgs_server, C.c_int64, C.POINTER(dgs_request_info)]),
    "dgs_server_wait": (C.c_int, [dgs_server, C.c_int64, C.c_double, C.POINTER(dgs_request_info)]),
    "dgs_server_cancel": (C.c_int, [dgs_server, C.c_int64]),
    "dgs_server_release": (C.c_int, [dgs_server, C.c_int64]),
    "dgs_server_get_stats": (C.c_int, [dgs_server, C.POINTER(dgs_server_stats)]),
    "dgs_server_last_error": (C.c_char_p, [dgs_server]),
    "dgs_server_destroy": (C.c_int, [dgs_server]),
}

DGS_NUM_STAGES = 9
STAGE_NAMES = ["cell_preprocess", "gauss_project", "depth_sort", "scan_emit", "tile_sort", "tile_ranges",
               "tile_depth_order", "work_queue", "composite"]

_lib = None


def lib():
    """The loaded libduplexgs.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                               "(python -m paper_2508_03180_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


class DgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status, ctx=None):
    if status != DGS_OK:
        msg = lib().dgs_last_error(ctx).decode() if ctx else ""
        raise DgsError(status, msg)
    return status


# C names, re-exported
def dgs_default_opts(opts):
    lib().dgs_default_opts(C.byref(opts))


def dgs_create(device, stream):
    h = dgs_ctx()
    check(lib().dgs_create(int(device), C.c_void_p(stream), C.byref(h)))
    return h


def dgs_destroy(ctx):
    return lib().dgs_destroy(ctx)


def dgs_set_stream(ctx, stream):
    return check(lib().dgs_set_stream(ctx, C.c_void_p(stream)), ctx)


def dgs_reserve(ctx, max_keys, max_prims, max_tiles):
    return check(lib().dgs_reserve(ctx, int(max_keys), int(max_prims), int(max_tiles)), ctx)


def dgs_render(ctx, scene, cam, opts, image, saved=None):
    """saved: None, or a dgs_frame() that receives the saved-frame handle."""
    return lib().dgs_render(ctx, C.byref(scene), C.byref(cam), C.byref(opts), C.byref(image),
                            C.byref(saved) if saved is not None else None)


def dgs_render_backward(ctx, scene, cam, opts, frame, grad_color_ptr, grad_weight_sum_ptr, grads):
    """cam / opts may be None (the frame's own)."""
    return lib().dgs_render_backward(ctx, C.byref(scene), C.byref(cam) if cam is not None else None,
                                     C.byref(opts) if opts is not None else None, frame,
                                     C.c_void_p(grad_color_ptr), C.c_void_p(grad_weight_sum_ptr), C.byref(grads))


def dgs_frame_release(ctx, frame):
    return lib().dgs_frame_release(ctx, frame)


def dgs_frame_stats(ctx, frame):
    s = dgs_stats()
    check(lib().dgs_frame_stats(ctx, frame, C.byref(s)), ctx)
    return s


def dgs_render_neural(ctx, scene, decoder, cam, opts, image):
    return lib().dgs_render_neural(ctx, C.byref(scene), C.byref(decoder), C.byref(cam), C.byref(opts),
                                   C.byref(image))


def dgs_read_decoded(ctx, means_ptr, scales_ptr, rots_ptr, opac_ptr, colors_ptr):
    return check(lib().dgs_read_decoded(ctx, C.c_void_p(means_ptr), C.c_void_p(scales_ptr), C.c_void_p(rots_ptr),
                                        C.c_void_p(opac_ptr), C.c_void_p(colors_ptr)), ctx)


def dgs_sync(ctx):
    return lib().dgs_sync(ctx)


def dgs_get_stats(ctx):
    s = dgs_stats()
    check(lib().dgs_get_stats(ctx, C.byref(s)), ctx)
    return s


def dgs_last_error(ctx):
    return lib().dgs_last_error(ctx).decode()


def dgs_read_lists(ctx, keys_ptr, values_ptr, ranges_ptr):
    return check(lib().dgs_read_lists(ctx, C.c_void_p(keys_ptr), C.c_void_p(values_ptr),
                                      C.c_void_p(ranges_ptr)), ctx)


def dgs_read_prims(ctx, rect_ptr, depth_ptr, ntiles_ptr):
    return check(lib().dgs_read_prims(ctx, C.c_void_p(rect_ptr), C.c_void_p(depth_ptr), C.c_void_p(ntiles_ptr)),
                 ctx)


def dgs_read_gauss_rects(ctx, rect_ptr):
    return check(lib().dgs_read_gauss_rects(ctx, C.c_void_p(rect_ptr)), ctx)


def dgs_sort_pairs(ctx, keys_ptr, values_ptr, n, key_bits):
    return check(lib().dgs_sort_pairs(ctx, C.c_void_p(keys_ptr), C.c_void_p(values_ptr), int(n), int(key_bits)),
                 ctx)


DGS_SORT_NOALLOC_MAX_KEYS = 1 << 20


def dgs_loss_l1_ssim(ctx, image_ptr, target_ptr, channels, height, width, lam, loss_ptr, grad_ptr):
    """(1 - lam) l1 + lam (1 - SSIM) of two planar images and dL/dimage
    (grad_ptr 0: the loss alone); all device pointers."""
    return lib().dgs_loss_l1_ssim(ctx, C.c_void_p(image_ptr), C.c_void_p(target_ptr), int(channels), int(height),
                                  int(width), float(lam), C.c_void_p(loss_ptr), C.c_void_p(grad_ptr or None))


def dgs_sort_pairs_noalloc(ctx, keys_ptr, values_ptr, n, key_bits):
    """Returns the status (no raise): callers check DGS_ERR_INVALID_ARG for n above the maximum."""
    return lib().dgs_sort_pairs_noalloc(ctx, C.c_void_p(keys_ptr), C.c_void_p(values_ptr), int(n), int(key_bits))


DGS_LIST_ORDER_AUTO, DGS_LIST_ORDER_PER_TILE, DGS_LIST_ORDER_GLOBAL = 0, 1, 2


def dgs_set_list_order(ctx, order):
    """Returns the status (no raise): invalid values give DGS_ERR_INVALID_ARG."""
    return lib().dgs_set_list_order(ctx, int(order))


def dgs_set_overlap(ctx, enable):
    return check(lib().dgs_set_overlap(ctx, int(bool(enable))), ctx)


def dgs_set_timing(ctx, enable):
    return check(lib().dgs_set_timing(ctx, int(bool(enable))), ctx)


def dgs_get_timing(ctx):
    ms = (C.c_float * DGS_NUM_STAGES)()
    frames = C.c_int32()
    check(lib().dgs_get_timing(ctx, ms, DGS_NUM_STAGES, C.byref(frames)), ctx)
    return list(ms), frames.value


# serving runtime
def dgs_server_default_config():
    cfg = dgs_server_config()
    lib().dgs_server_default_config(C.byref(cfg))
    return cfg


def server_check(status, srv):
    if status != DGS_OK:
        raise DgsError(status, lib().dgs_server_last_error(srv).decode() if srv else "")
    return status


def dgs_server_create(device, cfg):
    h = dgs_server()
    st = lib().dgs_server_create(int(device), C.byref(cfg), C.byref(h))
    if st != DGS_OK:
        raise DgsError(st, "server creation failed")
    return h


def dgs_server_create_simulated(cfg, sim):
    h = dgs_server()
    st = lib().dgs_server_create_simulated(C.byref(cfg), C.byref(sim), C.byref(h))
    if st != DGS_OK:
        raise DgsError(st, "simulated server creation failed")
    return h


def dgs_server_add_scene(srv, scene):
    sid = C.c_int32()
    server_check(lib().dgs_server_add_scene(srv, C.byref(scene), C.byref(sid)), srv)
    return sid.value


def dgs_server_submit(srv, scene_id, cam, opts, image):
    rid = C.c_int64()
    server_check(lib().dgs_server_submit(srv, int(scene_id), C.byref(cam), C.byref(opts) if opts is not None
                                         else None, C.byref(image), C.byref(rid)), srv)
    return rid.value


def dgs_server_query(srv, request_id):
    info = dgs_request_info()
    server_check(lib().dgs_server_query(srv, int(request_id), C.byref(info)), srv)
    return info


def dgs_server_wait(srv, request_id, timeout_s=-1.0):
    """The request's info once finished, or None on timeout."""
    info = dgs_request_info()
    st = lib().dgs_server_wait(srv, int(request_id), float(timeout_s), C.byref(info))
    if st == DGS_ERR_TIMEOUT:
        return None
    server_check(st, srv)
    return info


def dgs_server_cancel(srv, request_id):
    return lib().dgs_server_cancel(srv, int(request_id))


def dgs_server_release(srv, request_id):
    return lib().dgs_server_release(srv, int(request_id))


def dgs_server_get_stats(srv):
    s = dgs_server_stats()
    server_check(lib().dgs_server_get_stats(srv, C.byref(s)), srv)
    return s


def dgs_server_last_error(srv):
    return lib().dgs_server_last_error(srv).decode()


def dgs_server_destroy(srv):
    return lib().dgs_server_destroy(srv)
