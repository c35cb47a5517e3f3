#!/usr/bin/env python3
"""Frames per second of the Duplex-GS proxy-guided renderer on one MI355X.

Workload: the clustered 1M-Gaussian scene (100,000 cells x 10 Gaussians, SH
degree 3, seed 1) rendered at 1920x1080 along a 60-frame orbit, inputs
resident in HBM.  A step is one whole frame through the C ABI: cell
preprocess, Gaussian projection, depth sort of the cells, scan + key
emission, onesweep radix sort of the keys on their tile bits, tile ranges
and work queue, and the hybrid compositor.  The same frames are
also rendered by the per-Gaussian-sort alpha-blending path of the same
library (the comparison path).

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak (packed FP32: 2 lanes' worth per instruction)
# The compositor is compiled without packed-FP32 instructions, so the FP32
# rate its code can issue is 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA)
# x 2.4 GHz = 78.6 TFLOP/s; its roofline uses that peak.
PEAK_FP32_UNPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E

# Algorithmic FP32 work of the compositors (FMA counts 2), per counted event:
#   in-box evaluation: offsets (2), quadratic form (3 products, 3 multiply by
#   the conic, 2 adds), exp (1), times sigma (1)                       = 12
#   Duplex accumulated member: clamp (1), A (3 FMA = 6), B (1),
#   1 - v alpha (2), P *= (1)                                         = 11
#   Duplex blended cell per pixel: w = v T (1), N, D (4 FMA = 8), T *= P (1) = 10
#   alpha blended Gaussian: clamp (1), w = alpha T (1), C (3 FMA = 6),
#   T -= w (1)                                                         = 9
# lane operations per second of the FP32 vector units without packing
# (256 CUs x 64 lanes x 2.4 GHz) and of the transcendental unit (a quarter
# of that): the survey's per-lane work model of the compositor
LANE_OPS_PEAK = 256 * 64 * 2.4e9
EXP_PEAK = LANE_OPS_PEAK / 4
FLOP_BOX = 12
FLOP_DUPLEX_MEMBER = 11
FLOP_DUPLEX_CELL = 10
FLOP_ALPHA_HIT = 9

def tile_sort_passes(tiles):
    return (max(1, (tiles - 1).bit_length()) + 7) // 8


def sort_traffic(prims, keys, tiles, per_tile):
    """Algorithmic bytes of the sort: the passes over the (tile, depth) keys
    on their tile bits (u64 key + u32 value read and written: 24 B per key
    and pass), and either the depth order of the primitives before them --
    depth keys written (key and value, 8 B per primitive) and four 8-bit
    passes over them (16 B read and written per primitive and pass) -- or,
    with the per-tile order, the sort of each tile's run after them (24 B
    per key)."""
    tile_bytes = keys * 24 * tile_sort_passes(tiles)
    return tile_bytes + (keys * 24 if per_tile else prims * (8 + 4 * 16))


def sort_stage_ms(st):
    """The sort's stages: depth order of the primitives, tile sort, per-tile
    depth order (one of the depth stages is empty)."""
    return st["depth_sort"] + st["tile_sort"] + st["tile_depth_order"]


# algorithmic bytes of the Gaussian projection, per projected Gaussian:
# reads mean 12, scales 12, quaternion 16, opacity 4, SH (deg 3) 192,
# writes the 48-byte record and the 8-byte packed rectangle
BYTES_PROJECT_SH3 = 12 + 12 + 16 + 4 + 192 + 48 + 8

# HBM traffic of one Duplex compositor launch on this workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) scaled by a 1 GiB copy
# kernel's reading (profiles/composite_traffic_1080p_1M_pmc.md): 200.352 MB
# read + 51.105 MB written.  Valid for the compositor sources it was taken
# on; reported as null once one of them changes.
COMPOSITE_TRAFFIC_BYTES = 200.352e6 + 51.105e6
COMPOSITE_TRAFFIC_SOURCES = {
    "paper_2508_03180_amd/csrc/composite.hip": "9b908b67f959c8916ad4c0dcc83857436caea24a95f6f3b7a36644380df5d4dc",
    "paper_2508_03180_amd/csrc/common.h": "ba55af4abcd758f5c95eae4b782ec45303dc4fdba45ac22ae5f538575a823139",
    "paper_2508_03180_amd/csrc/cells.h": "462a33024d920aee0b8df89a3c7d1e57d0c202a65220e8a5e209d45b9729cb2d",
}


def composite_traffic():
    """Measured bytes per compositor launch, or None if the kernel changed."""
    import hashlib
    for rel, digest in COMPOSITE_TRAFFIC_SOURCES.items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    return COMPOSITE_TRAFFIC_BYTES


def progress(msg):
    """One line on stderr as each part of the run completes (stdout carries
    only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=120)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--frames-in-flight", type=int, default=3,
                   help="renderers (contexts on their own streams) taking the frames in turn in the extra "
                        "frames-in-flight leg; 0 skips it (the headline is one renderer)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-alpha", action="store_true")
    p.add_argument("--cpu-frames", type=int, default=3)
    p.add_argument("--bwd-steps", type=int, default=10)
    p.add_argument("--no-neural", action="store_true")
    p.add_argument("--no-ablation", action="store_true")
    p.add_argument("--no-ksweep", action="store_true")
    p.add_argument("--ksweep-frames", type=int, default=20)
    p.add_argument("--no-large", action="store_true")
    p.add_argument("--large-cams", type=int, default=20, help="cameras of each kind (near, far) per resolution")
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--serve-seconds", type=float, default=30.0, help="length of each Poisson stream")
    p.add_argument("--serve-rates", default="30,120,480", help="request rates (req/s)")
    p.add_argument("--serve-slots", type=int, default=4)
    p.add_argument("--serve-budget-gb", type=float, default=16.0, help="workspace budget of the server")
    return p.parse_args()


def differentiation(r, scene, cam, steps):
    """Forward + loss + backward through the planar autograd Function (the
    parameters are planar leaf tensors used in place) and the library's
    l1 + SSIM loss, with the render, the loss and the backward timed apart
    by HIP events on the torch stream."""
    import numpy as np
    import torch

    from paper_2508_03180_amd.renderer import DeviceScene, DuplexRenderPlanar, L1SsimLoss

    rng = np.random.default_rng(3)
    pert = dict(scene)
    pert["means"] = (scene["means"] + rng.normal(0, 0.01, scene["means"].shape)).astype(np.float32)
    logit = np.log(scene["opacities"] / (1 - scene["opacities"]))
    pert["opacities"] = (1 / (1 + np.exp(-(logit + rng.normal(0, 0.3, logit.shape))))).astype(np.float32)
    target = r.render(DeviceScene.from_numpy(pert, "cuda:0"), cam)["color"].clone()
    keys = ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "means", "scales", "rots", "opacities", "sh")
    ds = DeviceScene.from_numpy(scene, "cuda:0")
    pl = {k: ds.t[k].clone().requires_grad_(k not in ("cell_scale", "cell_rot")) for k in keys}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(timed):
        for v in pl.values():
            v.grad = None
        if timed:
            ev[0].record()
        C, _ = DuplexRenderPlanar.apply(r, cam, {}, *[pl[k] for k in keys])
        if timed:
            ev[1].record()
        loss = L1SsimLoss.apply(r, C, target, 0.2)
        if timed:
            ev[2].record()
        loss.backward()
        if timed:
            ev[3].record()
        return loss

    for _ in range(3):
        step(False)
    torch.cuda.synchronize()
    parts = np.zeros(3)
    t0 = time.perf_counter()
    for _ in range(steps):
        loss = step(True)
        torch.cuda.synchronize()
        parts += [ev[i].elapsed_time(ev[i + 1]) for i in range(3)]
    dt = (time.perf_counter() - t0) / steps
    parts /= steps
    # the library's backward alone (composite and projection backward kernels)
    from paper_2508_03180_amd import _capi as capi
    out = r.render(ds, cam, save=True)
    gC = torch.randn_like(out["color"])
    r.render_backward(ds, out["frame"], gC)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        r.render_backward(ds, out["frame"], gC)
    e1.record()
    torch.cuda.synchronize()
    bt = e0.elapsed_time(e1) / steps
    out.pop("frame").release()
    capi.check(capi.dgs_sync(r.ctx), r.ctx)
    return {"loss": "0.8 L1 + 0.2 (1 - SSIM 11x11), library kernels, vs perturbed-scene target",
            "width": 1920, "height": 1080,
            "params": "planar leaf tensors (no layout copies)",
            "fwd_loss_bwd_ms": round(dt * 1e3, 3), "render_ms": round(float(parts[0]), 3),
            "loss_ms": round(float(parts[1]), 3), "loss_and_render_backward_ms": round(float(parts[2]), 3),
            "backward_ms": round(bt, 3), "final_loss": round(float(loss.detach()), 5)}


# LC-WSR weights of the "w/o T^cell" variant on the mid scene: the farthest
# cell of the orbit sits at depth ~5.6, so weights fall linearly from ~0.8 in
# front to ~0.3 at the back and none is clamped to 0
ABLATION_TAU = 8.0


def ablation(r, ds, cams, timed_frames):
    """Frames/s of the variants of the ablation table on the benchmark orbit:
    the full method, w/o T^cell (LC-WSR cell weights), w/o ET, w/o v_n."""
    import torch
    variants = {"full": {}, "wo_Tcell": dict(mode="lcwsr", tau=ABLATION_TAU), "wo_ET": dict(no_et=True),
                "wo_v": dict(v_one=True)}
    out = {}
    for name, kw in variants.items():
        nval = nrend = 0
        for c in cams[::6]:
            r.render(ds, c, **kw, stats=True)
            st = r.stats()
            nval += st["n_val"]
            nrend += st["n_rendered"]
        img = r.alloc_image(cams[0])
        for c in cams[:5]:
            r.render(ds, c, out=img, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(timed_frames):
            r.render(ds, cams[i % len(cams)], out=img, check=False, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert r.sync() == 0
        out[name] = {"fps": round(timed_frames / dt, 2), "termination_ratio": round(1 - nrend / max(nval, 1), 4),
                     "rendered_per_pixel": round(nrend / len(cams[::6]) / (cams[0]["width"] * cams[0]["height"]), 3)}
    out["tau"] = ABLATION_TAU
    return out


def neural(a, cams, steps):
    """The neural variant of the mid scene (100,000 cells x 10, features 32,
    hidden 32, random decoder weights): frames/s of the whole frame
    including the decode of the visible cells, and the decode's share."""
    import torch

    from paper_2508_03180_amd import _capi as capi
    from paper_2508_03180_amd import scenes
    from paper_2508_03180_amd.renderer import NeuralDeviceScene, Renderer

    s, d = scenes.make_neural_scene(1)
    ns = NeuralDeviceScene.from_numpy(s, d, "cuda:0")
    r = Renderer(0)
    img = r.alloc_image(cams[0])
    for c in cams[:10]:
        r.render_neural(ns, c, out=img)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        r.render_neural(ns, cams[i % len(cams)], out=img, check=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert r.sync() == 0
    capi.dgs_set_timing(r.ctx, 1)
    for c in cams:
        r.render_neural(ns, c, out=img, check=False)
    ms, nfr = capi.dgs_get_timing(r.ctx)
    capi.dgs_set_timing(r.ctx, 0)
    st = {k: round(v / nfr, 4) for k, v in zip(capi.STAGE_NAMES, ms)}
    r.close()
    macs = 0
    F, H, K = d["F"], d["H"], s["K"]
    for a_ in (1, 3, 3, 4):
        macs += (F + 4) * H + H * K * a_
    return {"fps": round(steps / dt, 2), "feature_dim": F, "hidden_dim": H,
            "decode_macs_per_cell": macs,
            "stages_ms": st, "note": "stage cell_preprocess includes the decode of the visible cells"}


KSWEEP = (1, 2, 5, 10, 20, 32)


def k_sweep(a):
    """Members per cell K at a fixed 1M Gaussians (mid-scene generator with
    1M / K cells), 1080p orbit: keys, cells in the frustum, valid Gaussians
    per pixel and frames/s of both modes."""
    import torch

    from paper_2508_03180_amd import scenes
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer

    cams = scenes.orbit_cameras(60, 1920, 1080)[::60 // a.ksweep_frames][:a.ksweep_frames]
    r = Renderer(0)
    out = {"gaussians": 1_000_000, "frames": len(cams)}
    for K in KSWEEP:
        ds = DeviceScene.from_numpy(scenes.make_mid_scene(1, n_cells=1_000_000 // K, K=K), "cuda:0")
        img = r.alloc_image(cams[0])
        res = {}
        for mode in ("duplex", "alpha"):
            keys = nval = vis = 0
            for c in cams:
                r.render(ds, c, out=img, mode=mode, stats=True)
                st = r.stats()
                keys += st["num_keys"]
                nval += st["n_val"]
                if mode == "duplex":
                    _, _, nt = r.read_prims(ds.N)
                    vis += int((nt > 0).sum().item())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in cams:
                r.render(ds, c, out=img, mode=mode, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            assert r.sync() == 0
            res[mode] = {"fps": round(len(cams) / dt, 2), "keys_mean": round(keys / len(cams), 1),
                         "valid_per_pixel": round(nval / len(cams) / (1920 * 1080), 3)}
            if mode == "duplex":
                res[mode]["cells_in_frustum"] = round(vis / len(cams), 1)
        res["speedup"] = round(res["duplex"]["fps"] / res["alpha"]["fps"], 3)
        out[f"K{K}"] = res
        del ds, img
    r.close()
    torch.cuda.empty_cache()
    return out


LARGE_SIZES = [(1280, 720), (1920, 1080), (3840, 2160)]


def large_scene(a):
    """6M-Gaussian aerial-scale scene (600k cells x 10) at 720p, 1080p and 4K
    over near and far cameras: sort-key reduction of per-cell keys against
    per-Gaussian keys, the early-termination rate 1 - sum N^rendered / sum
    N^val, and frames/s of both modes."""
    import numpy as np
    import torch

    from paper_2508_03180_amd import scenes
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer

    scene = scenes.make_large_scene(2)
    ds = DeviceScene.from_numpy(scene, "cuda:0")
    del scene
    r = Renderer(0)
    out = {"gaussians": ds.M, "cells": ds.N, "cameras_per_kind": a.large_cams}
    for (w, h) in LARGE_SIZES:
        allc = scenes.large_scene_cameras(2, w, h, n_near=20, n_far=20)
        cams = allc[:a.large_cams] + allc[20:20 + a.large_cams]
        img = r.alloc_image(cams[0])
        res = {}
        for mode in ("duplex", "alpha"):
            keys = nval = nrend = 0
            for c in cams:  # sizes the workspace and counts
                r.render(ds, c, out=img, mode=mode, stats=True)
                st = r.stats()
                keys += st["num_keys"]
                nval += st["n_val"]
                nrend += st["n_rendered"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in cams:
                r.render(ds, c, out=img, mode=mode, check=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            capi_check = r.sync()
            assert capi_check == 0, capi_check
            res[mode] = {"fps": round(len(cams) / dt, 2), "keys_mean": round(keys / len(cams), 1),
                         "termination_ratio": round(1 - nrend / max(nval, 1), 4)}
        res["key_reduction"] = round(1 - res["duplex"]["keys_mean"] / res["alpha"]["keys_mean"], 4)
        res["speedup"] = round(res["duplex"]["fps"] / res["alpha"]["fps"], 3)
        out[f"{w}x{h}"] = res
        del img
    r.close()
    del ds
    torch.cuda.empty_cache()
    return out


SERVE_SIZES = [(640, 480), (1280, 720), (1920, 1080), (3840, 2160)]


def serving(a):
    """Serving load: four scenes (200k, 1M, 3M, 6M Gaussians), resolution
    uniform over SERVE_SIZES, Poisson arrivals at each rate; the native server
    (frames in flight on several streams, graph replay, memory budget)
    against one-at-a-time serving (one slot, direct launches) on the same
    request stream."""
    import numpy as np

    from paper_2508_03180_amd import scenes
    from paper_2508_03180_amd.renderer import DeviceScene
    from paper_2508_03180_amd.serving import Server, poisson_schedule, run_load, run_saturated

    gen = [lambda: scenes.make_mid_scene(40, n_cells=20_000), lambda: scenes.make_mid_scene(41),
           lambda: scenes.make_large_scene(42, n_cells=300_000), lambda: scenes.make_large_scene(43)]
    ds = []
    for g in gen:
        ds.append(DeviceScene.from_numpy(g(), "cuda:0"))
    ncam = 12
    cams = {}
    for i in range(4):
        cams[i] = {}
        for (w, h) in SERVE_SIZES:
            if i < 2:
                cams[i][(w, h)] = scenes.orbit_cameras(ncam, w, h, step_deg=30.0)
            else:
                cams[i][(w, h)] = scenes.aerial_orbit_cameras(ncam, w, h, step_deg=30.0)
    rates = [float(x) for x in a.serve_rates.split(",") if x]
    warm = poisson_schedule(1000.0, 0.25, 4, cams, seed=7)
    sat = poisson_schedule(1000.0, 0.3, 4, cams, seed=8)
    out = {"scenes_gaussians": [d.M for d in ds], "sizes": [f"{w}x{h}" for w, h in SERVE_SIZES],
           "seconds_per_rate": a.serve_seconds, "budget_gb": a.serve_budget_gb}
    configs = {"server": dict(num_slots=a.serve_slots, use_graphs=True,
                              memory_budget=int(a.serve_budget_gb * (1 << 30))),
               "one_at_a_time": dict(num_slots=1, use_graphs=False, memory_budget=0)}
    for name, kw in configs.items():
        with Server(0, **kw) as srv:
            ids = [srv.add_scene(d) for d in ds]
            run_saturated(srv, ids, warm)  # captures graphs, learns key counts
            res = {"saturated_frames_per_s": round(run_saturated(srv, ids, sat), 2)}
            for k, rate in enumerate(rates):
                sched = poisson_schedule(rate, a.serve_seconds, 4, cams, seed=100 + k)
                res[f"{int(rate)}"] = {kk: (round(v, 4) if isinstance(v, float) else v)
                                       for kk, v in run_load(srv, ids, sched, rate).summary().items()}
                progress(f"serving {name} at {rate:g} req/s: p99 {res[f'{int(rate)}'].get('p99_ms')} ms")
            st = srv.stats()
            res["stats"] = {k: st[k] for k in ("completed", "failed", "retries", "graph_captures",
                                               "graph_replays", "releases", "peak_workspace_bytes")}
        out[name] = res
    for k in [f"{int(r)}" for r in rates]:
        s, o = out["server"][k], out["one_at_a_time"][k]
        out[f"p99_speedup_{k}"] = round(o["p99_ms"] / s["p99_ms"], 3) if s["p99_ms"] else None
    out["throughput_speedup"] = round(out["server"]["saturated_frames_per_s"]
                                      / out["one_at_a_time"]["saturated_frames_per_s"], 3)
    return out


def cpu_baseline(scene, cams, nframes):
    """The oracle (plain CPU reference, not an optimised renderer) timed on
    the host: the headline value is full 1080p frames of the benchmark's
    workload on every host thread; also one frame on one thread, the
    per-Gaussian alpha-blend oracle on one frame, the tiny scene (median of
    three) and two street-level plus two aerial 720p views of the large
    scene."""
    import numpy as np

    import oracle
    from paper_2508_03180_amd import scenes

    allc = oracle.num_threads()

    def per_frame(fn, reps=1):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    idx = [0, 20, 40][:nframes]
    t = sum(per_frame(lambda i=i: oracle.render(scene, cams[i])) for i in idx)
    out = {"value": round(len(idx) / t, 4), "unit": "frames/s", "cores": allc, "kind": "oracle",
           "sample": f"{len(idx)} full 1920x1080 frames (orbit frames {idx}) of the benchmark scene, "
                     f"Duplex oracle on {allc} threads"}
    out["alpha_oracle_frame_s"] = round(per_frame(lambda: oracle.render(scene, cams[0], mode="alpha")), 3)
    tiny, tcam = scenes.make_tiny_scene(0), scenes.tiny_camera()
    out["tiny_frame_ms"] = round(1e3 * per_frame(lambda: oracle.render(tiny, tcam), 3), 2)
    large = scenes.make_large_scene(2)
    lc = scenes.large_scene_cameras(2, 1280, 720, n_near=20, n_far=20)
    out["large_720p_frame_s"] = round(np.mean([per_frame(lambda c=c: oracle.render(large, c))
                                               for c in (lc[0], lc[1], lc[20], lc[21])]), 3)
    del large
    oracle.set_threads(1)
    try:
        out["one_core"] = {"frame_s": round(per_frame(lambda: oracle.render(scene, cams[0])), 3),
                           "tiny_frame_ms": round(1e3 * per_frame(lambda: oracle.render(tiny, tcam), 3), 2)}
    finally:
        oracle.set_threads(allc)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this renderer runs on one GPU; multi-GPU runs are not supported (--gpus 1)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2508_03180_amd import _capi as capi
    from paper_2508_03180_amd import scenes
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer, camera_struct, opts_struct

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    W, H, NF = 1920, 1080, 60
    TILES = ((W + 15) // 16) * ((H + 15) // 16)
    scene = scenes.make_mid_scene(1)
    cams = scenes.orbit_cameras(NF, W, H)
    r = Renderer(0)
    ds = DeviceScene.from_numpy(scene, "cuda:0")
    out = r.alloc_image(cams[0])
    cam_structs = [camera_struct(c) for c in cams]
    sc = ds.struct()
    im = capi.dgs_image()
    im.color, im.weight_sum = out["color"].data_ptr(), out["D"].data_ptr()
    im.final_T, im.last = out["T"].data_ptr(), out["last"].data_ptr()
    L = capi.lib()

    def frames(mode, n):
        op = opts_struct(mode=mode)
        for i in range(n):
            st = L.dgs_render(r.ctx, sc, cam_structs[i % NF], op, im, None)
            if st:
                capi.check(st, r.ctx)

    def size_all(mode):
        keys = []
        for i in range(NF):
            r.render(ds, cams[i], out=out, mode=mode)
            keys.append(r.stats()["num_keys"])
        return keys

    def timed(mode, steps, warmup):
        frames(mode, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        frames(mode, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        capi.check(capi.dgs_sync(r.ctx), r.ctx)
        return dt

    # frames in flight: F renderers, each a context on its own stream with its
    # own workspace and output image, take the orbit frames in turn, so one
    # frame's sort can run beside another's compositor.  Every frame is still
    # rendered whole; in-frame overlap is off (one stream per context).
    F = max(0, a.frames_in_flight)
    flight = []
    for _ in range(F):
        rr = Renderer(0, stream=torch.cuda.Stream(), overlap=(F == 1))
        oo = rr.alloc_image(cams[0])
        flight.append((rr, oo, capi.dgs_image(oo["color"].data_ptr(), oo["D"].data_ptr(), oo["T"].data_ptr(),
                                              oo["last"].data_ptr())))

    def timed_in_flight(mode, steps, warmup):
        op = opts_struct(mode=mode)
        for rr, oo, _ in flight:  # size every workspace for the whole orbit
            for c in cams:
                rr.render(ds, c, out=oo, mode=mode)
        torch.cuda.synchronize()

        def go(first, n):
            for i in range(first, first + n):
                rr, _, ii = flight[i % F]
                st = L.dgs_render(rr.ctx, sc, cam_structs[i % NF], op, ii, None)
                if st:
                    capi.check(st, rr.ctx)

        go(-warmup, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        go(0, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        for j, (rr, oo, _) in enumerate(flight):
            capi.check(capi.dgs_sync(rr.ctx), rr.ctx)
            done = [i for i in range(steps) if i % F == j]
            if done:  # the renderer's last frame is the frame rendered alone
                ref = r.render(ds, cams[done[-1] % NF], out=out, mode=mode)["color"]
                torch.cuda.synchronize()
                assert torch.equal(oo["color"], ref), ("frames in flight changed a frame", mode, j)
        return dt

    def frame_times(mode, orbits=2):
        """Per-frame GPU time (HIP events between consecutive frames on the
        context stream) over the orbit: median, p99 and max in ms."""
        op = opts_struct(mode=mode)
        n = orbits * NF
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        ev[0].record(r.stream)
        for i in range(n):
            st = L.dgs_render(r.ctx, sc, cam_structs[i % NF], op, im, None)
            if st:
                capi.check(st, r.ctx)
            ev[i + 1].record(r.stream)
        torch.cuda.synchronize()
        ms = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(n)])
        return {"frames": n, "median_ms": round(float(np.median(ms)), 4),
                "p99_ms": round(float(np.percentile(ms, 99)), 4), "max_ms": round(float(ms.max()), 4)}

    def stage_times(mode):
        capi.dgs_set_timing(r.ctx, 1)
        frames(mode, NF)
        ms, nfr = capi.dgs_get_timing(r.ctx)
        capi.dgs_set_timing(r.ctx, 0)
        return {k: v / nfr for k, v in zip(capi.STAGE_NAMES, ms)}

    def counters(mode, idx):
        tot = dict(n_val=0, n_rendered=0, n_box=0, n_cell_hits=0, n_cell_pixels=0, keys=0, projected=0,
                   per_tile=0)
        for i in idx:
            r.render(ds, cams[i], out=out, mode=mode, stats=True)
            s = r.stats()
            for k in ("n_val", "n_rendered", "n_box", "n_cell_hits", "n_cell_pixels"):
                tot[k] += s[k]
            tot["keys"] += s["num_keys"]
            tot["per_tile"] += s["sort_passes"] == tile_sort_passes(TILES)  # no depth-sort passes
            if mode == "duplex":
                _, _, nt = r.read_prims(ds.N)
                tot["projected"] += int((nt > 0).sum().item()) * ds.K
            else:
                tot["projected"] += ds.M
        return {k: v / len(idx) for k, v in tot.items()}

    keys_dup = size_all("duplex")
    dt = timed("duplex", a.steps, a.warmup)
    fps = a.steps / dt
    dtf = timed_in_flight("duplex", a.steps, a.warmup) if F else None
    progress(f"duplex: {fps:.1f} frames/s" + (f", {a.steps / dtf:.1f} with {F} frames in flight" if F else ""))
    st_dup = stage_times("duplex")
    fr_dup = frame_times("duplex")
    cnt = counters("duplex", range(0, NF, 6))

    alpha = None
    if not a.no_alpha:
        keys_alpha = size_all("alpha")
        dta = timed("alpha", a.steps, a.warmup)
        dtaf = timed_in_flight("alpha", a.steps, a.warmup) if F else None
        st_alpha = stage_times("alpha")
        fr_alpha = frame_times("alpha")
        cnt_a = counters("alpha", range(0, NF, 6))
        progress(f"alpha-blend baseline: {a.steps / dta:.1f} frames/s")
        comp_a = st_alpha["composite"]
        flops_a = FLOP_BOX * cnt_a["n_box"] + FLOP_ALPHA_HIT * cnt_a["n_rendered"]
        alpha = {"fps": round(a.steps / dta, 2), "ms_per_step": round(1e3 * dta / a.steps, 4),
                 "frame_ms": fr_alpha,
                 "stages_ms": {k: round(v, 4) for k, v in st_alpha.items()},
                 "keys_mean": float(np.mean(keys_alpha)),
                 "composite_tflops": round(flops_a / (comp_a * 1e-3) / 1e12, 3),
                 "sort_ms": round(sort_stage_ms(st_alpha), 4),
                 "sort_keys_per_s": round(cnt_a["keys"] / (sort_stage_ms(st_alpha) * 1e-3), 1),
                 "sort_hbm_frac": round(sort_traffic(ds.M, cnt_a["keys"], TILES, cnt_a["per_tile"] > 0.5)
                                        / (sort_stage_ms(st_alpha) * 1e-3) / (PEAK_HBM_GBS * 1e9), 4),
                 "list_order": "per_tile" if cnt_a["per_tile"] > 0.5 else "global"}

    for rr, _, _ in flight:  # the later legs run on their own streams
        rr.close()
    flight.clear()

    # roofline of the dominant kernel, the Duplex compositor (plain FP32 ALU)
    comp_ms = st_dup["composite"]
    flops = (FLOP_BOX * cnt["n_box"] + FLOP_DUPLEX_MEMBER * cnt["n_rendered"]
             + FLOP_DUPLEX_CELL * cnt["n_cell_hits"])
    achieved = flops / (comp_ms * 1e-3) / 1e12
    # the survey's work terms: E in-box member-pixel evaluations (~16 lane
    # operations and one exp each), L listed member-pixel pairs (~4 for the
    # box test), cell-pixel pairs reached (~8 for the cell update)
    E, cp = cnt["n_box"], cnt["n_cell_pixels"]
    Lp = cp * ds.K
    lane_ops = 16 * E + 4 * Lp + 8 * cp
    t_s = comp_ms * 1e-3
    traffic = composite_traffic()  # measured HBM bytes per launch (None once the compositor changed)
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "peak_issuable_unpacked": round(PEAK_FP32_UNPACKED_TFLOPS, 2),
            "frac_of_issuable": round(achieved / PEAK_FP32_UNPACKED_TFLOPS, 4), "traffic": traffic,
            "traffic_gbs": round(traffic / t_s / 1e9, 1) if traffic else None,
            "traffic_hbm_frac": round(traffic / t_s / (PEAK_HBM_GBS * 1e9), 4) if traffic else None,
            "kernel": "k_composite<0, false, false, false>", "kernel_ms": round(comp_ms, 4),
            "algorithmic_gflop_per_launch": round(flops / 1e9, 4),
            "work_terms": {"E_inbox_member_pixels": int(E), "L_listed_member_pixels": int(Lp),
                           "cell_pixels": int(cp), "lane_ops_per_launch": int(lane_ops),
                           "lane_op_rate_T_per_s": round(lane_ops / t_s / 1e12, 3),
                           "lane_op_frac_of_39_3T": round(lane_ops / t_s / LANE_OPS_PEAK, 4),
                           "exp_rate_T_per_s": round(E / t_s / 1e12, 3),
                           "exp_frac_of_9_8T": round(E / t_s / EXP_PEAK, 4)}}
    proj_gbs = cnt["projected"] * BYTES_PROJECT_SH3 / (st_dup["gauss_project"] * 1e-3) / 1e9

    # differentiation: forward + 0.8 L1 + 0.2 (1 - SSIM) + backward at 1080p
    # against a target rendered from a perturbed copy of the scene
    bwd = differentiation(r, scene, cams[0], a.bwd_steps)
    progress(f"differentiation: {bwd['fwd_loss_bwd_ms']} ms per step")

    neu = None if a.no_neural else neural(a, cams, a.steps)
    progress("neural decode done")
    abl = None if a.no_ablation else ablation(r, ds, cams, a.steps)
    progress("ablation done")
    ksw = None if a.no_ksweep else k_sweep(a)
    progress("K sweep done")
    large = None if a.no_large else large_scene(a)
    progress("large scene done")
    serve = None if a.no_serve else serving(a)
    progress("serving done")

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(scene, cams, a.cpu_frames)
        progress("cpu baseline done")

    line = {
        "metric": "FPS @1080p, 1M Gaussians vs per-Gaussian-sort baseline; serve p50/p99 ms",
        "value": round(fps, 2), "unit": "frames/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(1e3 * dt / a.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "clustered scene, 100k cells x 10 Gaussians (1M), SH degree 3, "
                               "1920x1080, 60-frame orbit", "cells": ds.N, "gaussians": ds.M,
                   "width": W, "height": H, "frames": NF,
                   "timed_frames": f"orbit frames i mod {NF} for i = 0..{a.steps - 1} "
                                   f"({'the whole orbit' if a.steps >= NF else f'{a.steps} of {NF} frames'}), "
                                   f"after {a.warmup} untimed warm-up frames, back to back on one renderer"},
        "alpha_baseline": alpha,
        "speedup_vs_alpha": None if alpha is None else round(fps / alpha["fps"], 3),
        "frames_in_flight": None if not F else {
            "renderers": F, "note": "the same timed frames given in turn to renderers on their own streams; "
                                    "every frame rendered whole (not the headline protocol)",
            "fps": round(a.steps / dtf, 2), "ms_per_step": round(1e3 * dtf / a.steps, 4),
            "alpha_fps": None if alpha is None else round(a.steps / dtaf, 2),
            "speedup_vs_alpha": None if alpha is None else round(dtaf / dtf, 3)},
        "frame_ms": fr_dup,
        "stages_ms": {k: round(v, 4) for k, v in st_dup.items()},
        "keys_mean": float(np.mean(keys_dup)),
        "key_reduction_vs_alpha": None if alpha is None else round(1 - np.mean(keys_dup) / alpha["keys_mean"], 4),
        "sort_ms": round(sort_stage_ms(st_dup), 4),
        "sort_keys_per_s": round(cnt["keys"] / (sort_stage_ms(st_dup) * 1e-3), 1),
        "sort_hbm_frac": round(sort_traffic(ds.N, cnt["keys"], TILES, cnt["per_tile"] > 0.5)
                               / (sort_stage_ms(st_dup) * 1e-3) / (PEAK_HBM_GBS * 1e9), 4),
        "list_order": "per_tile" if cnt["per_tile"] > 0.5 else "global",
        "projection_hbm_gbs": round(proj_gbs, 1),
        "projection_hbm_frac": round(proj_gbs / PEAK_HBM_GBS, 4),
        "termination_ratio": round(1 - cnt["n_rendered"] / max(cnt["n_val"], 1), 4),
        "roofline": roof,
        "differentiation": bwd,
        "neural": neu,
        "ablation": abl,
        "k_sweep": ksw,
        "large_scene": large,
        "serving": serve,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    for rr, _, _ in flight:
        rr.close()
    r.close()


if __name__ == "__main__":
    main()
