"""Python driver of the native serving runtime (argument marshalling, output
allocation and a Poisson load generator).

The scheduler, admission control, graph capture and retries all run in the
library (dgs_server_* in include/duplexgs.h); this module only submits
requests, keeps their output tensors alive until they finish and summarises
latencies.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _capi as capi
from .renderer import DeviceScene, camera_struct, opts_struct

STATE_NAMES = {capi.DGS_REQ_QUEUED: "queued", capi.DGS_REQ_RUNNING: "running", capi.DGS_REQ_DONE: "done",
               capi.DGS_REQ_FAILED: "failed", capi.DGS_REQ_CANCELLED: "cancelled"}


def info_dict(info):
    return {k: getattr(info, k) for k, _ in capi.dgs_request_info._fields_ if k != "reserved"}


class Server:
    """A dgs_server on one device (or the simulated device when `simulate` is
    a dict with seconds_fixed / seconds_per_mpixel / keys_per_pixel)."""

    def __init__(self, device=0, num_slots=4, use_graphs=True, memory_budget=0, simulate=None):
        cfg = capi.dgs_server_default_config()
        cfg.num_slots = int(num_slots)
        cfg.use_graphs = int(bool(use_graphs))
        cfg.memory_budget = int(memory_budget)
        if simulate is not None:
            sim = capi.dgs_sim_device(float(simulate.get("seconds_fixed", 0.0)),
                                      float(simulate.get("seconds_per_mpixel", 0.0)),
                                      float(simulate.get("keys_per_pixel", 0.0)))
            self.h = capi.dgs_server_create_simulated(cfg, sim)
            self.device = None
        else:
            self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
            self.h = capi.dgs_server_create(self.device.index or 0, cfg)
        self._scenes = []   # keeps scene memory alive
        self._outputs = {}  # request id -> output tensors (alive until finished)
        self._lock = threading.Lock()

    # -- scenes and requests
    def add_scene(self, scene):
        """scene: a DeviceScene (or a raw capi.dgs_scene for the simulated device)."""
        st = scene.struct() if isinstance(scene, DeviceScene) else scene
        sid = capi.dgs_server_add_scene(self.h, st)
        self._scenes.append(scene)
        return sid

    def submit(self, scene_id, cam, out=None, image=None, **opts):
        """Queues one frame; returns its request id.  The colour image
        ([3][H][W] float32) is allocated unless `out` (a tensor) or `image`
        (a capi.dgs_image, e.g. for the simulated device) is given."""
        if image is None:
            if out is None:
                out = torch.empty((3, int(cam["height"]), int(cam["width"])), dtype=torch.float32,
                                  device=self.device)
            image = capi.dgs_image(out.data_ptr(), None, None, None)
        rid = capi.dgs_server_submit(self.h, scene_id, camera_struct(cam), opts_struct(**opts), image)
        if out is not None:
            with self._lock:
                self._outputs[rid] = out
        return rid

    def query(self, rid):
        return info_dict(capi.dgs_server_query(self.h, rid))

    def wait(self, rid, timeout=None, release=True):
        """(info dict, colour tensor or None); raises TimeoutError."""
        info = capi.dgs_server_wait(self.h, rid, -1.0 if timeout is None else float(timeout))
        if info is None:
            raise TimeoutError(f"request {rid} not finished")
        with self._lock:
            out = self._outputs.pop(rid, None) if release else self._outputs.get(rid)
        if release:
            capi.dgs_server_release(self.h, rid)
        return info_dict(info), out

    def cancel(self, rid):
        return capi.dgs_server_cancel(self.h, rid) == capi.DGS_OK

    def stats(self):
        s = capi.dgs_server_get_stats(self.h)
        return {k: getattr(s, k) for k, _ in capi.dgs_server_stats._fields_}

    def last_error(self):
        return capi.dgs_server_last_error(self.h)

    def close(self):
        if self.h:
            capi.dgs_server_destroy(self.h)
            self.h = None
            self._outputs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- load

@dataclass
class LoadResult:
    rate: float
    n: int
    latencies_ms: np.ndarray
    span_s: float
    failed: int
    submit_lag_ms: np.ndarray
    stats: dict = field(default_factory=dict)

    def summary(self):
        lat = self.latencies_ms
        return {
            "rate_req_s": self.rate,
            "requests": self.n,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "frames_per_s": float(lat.size / self.span_s) if self.span_s > 0 else None,
            "failed": self.failed,
            "submit_lag_p99_ms": float(np.percentile(self.submit_lag_ms, 99)) if self.submit_lag_ms.size else None,
        }


def poisson_schedule(rate, duration, n_scenes, cams, seed):
    """Arrival times (s), scene ids and camera picks of a Poisson stream:
    scene uniform, resolution uniform over cams[scene] keys, camera uniform
    over that list."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        s = int(rng.integers(n_scenes))
        res_keys = sorted(cams[s])
        res = res_keys[int(rng.integers(len(res_keys)))]
        cam = cams[s][res][int(rng.integers(len(cams[s][res])))]
        out.append((t, s, cam))
    return out


def run_load(server, scene_ids, schedule, rate, **opts):
    """Submits `schedule` in real time and waits for every request.  Latency
    is completion minus submission on the server's clock."""
    ids = []
    lag = []
    done = []
    failed = [0]

    def waiter():
        i = 0
        while True:
            while i >= len(ids):
                if finished_submitting.is_set() and i >= len(ids):
                    return
                time.sleep(0.0005)
            info, _ = server.wait(ids[i])
            if info["state"] == capi.DGS_REQ_DONE:
                done.append((info["t_submit"], info["t_done"]))
            else:
                failed[0] += 1
            i += 1

    finished_submitting = threading.Event()
    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for (t, s, cam) in schedule:
        now = time.perf_counter() - t0
        if t > now:
            time.sleep(t - now)
        lag.append((time.perf_counter() - t0 - t) * 1e3)
        ids.append(server.submit(scene_ids[s], cam, **opts))
    finished_submitting.set()
    th.join()
    if done:
        ts = np.array(done)
        lat = (ts[:, 1] - ts[:, 0]) * 1e3
        span = float(ts[:, 1].max() - ts[:, 0].min())
    else:
        lat, span = np.zeros(0), 0.0
    return LoadResult(rate, len(schedule), lat, span, failed[0], np.array(lag), server.stats())


def run_saturated(server, scene_ids, schedule, **opts):
    """Submits every request at once and returns frames/s over the batch."""
    t0 = time.perf_counter()
    ids = [server.submit(scene_ids[s], cam, **opts) for (_, s, cam) in schedule]
    infos = [server.wait(i)[0] for i in ids]
    t1 = time.perf_counter()
    ok = sum(1 for i in infos if i["state"] == capi.DGS_REQ_DONE)
    return ok / (t1 - t0)
