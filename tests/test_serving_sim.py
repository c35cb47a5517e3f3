"""Scheduler, admission and retry logic of the native serving runtime, on the
library's simulated device (host only: nothing is allocated on a GPU and no
scene or image pointer is dereferenced, so fake addresses stand in)."""
import threading
import time

import numpy as np
import pytest

from paper_2508_03180_amd import _capi as capi
from paper_2508_03180_amd import scenes
from paper_2508_03180_amd.serving import Server, poisson_schedule, run_load

FAKE = 0x10000


def fake_scene(n_cells=1000, K=10, cells=True):
    s = capi.dgs_scene()
    s.num_cells, s.gaussians_per_cell = n_cells, K
    for k in ("means", "scales", "rots", "opacities", "sh"):
        setattr(s, k, FAKE)
    if cells:
        for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh"):
            setattr(s, k, FAKE)
    s.v_sh_degree, s.sh_degree = 1, 0
    return s


def image():
    return capi.dgs_image(FAKE, None, None, None)


def cam(w, h):
    return scenes.pinhole(scenes.look_at((0, 0, 3), (0, 0, 0)), w, h)


def sim_server(slots=4, graphs=True, budget=0, fixed=0.0, per_mpx=0.01, keys_per_px=0.1):
    return Server(num_slots=slots, use_graphs=graphs, memory_budget=budget,
                  simulate=dict(seconds_fixed=fixed, seconds_per_mpixel=per_mpx, keys_per_pixel=keys_per_px))


def bytes_for(prims, gauss, keys, tiles):
    """Workspace bytes of a context at these capacities (the library's
    accounting: 40 B per primitive (depth, rectangle, tile count, offset, v,
    and the depth sort's keys and values twice) + 8 B per 2048-primitive scan
    partition (+ 8) + 256 x 8 B per 1024-primitive sort partition, 56 B per
    Gaussian, 24 B per key + 256 x 8 B per 1024-key sort partition, 24 B per
    tile)."""
    b = 0
    if prims:
        b += prims * 40 + ((prims + 2047) // 2048 + 1) * 8 + ((prims + 1023) // 1024) * 256 * 8
    if gauss:
        b += gauss * 56
    if keys:
        b += keys * 24 + ((keys + 1023) // 1024) * 256 * 8
    if tiles:
        b += tiles * 24
    return b


def test_all_requests_complete_in_order_with_one_slot():
    with sim_server(slots=1, fixed=0.002) as srv:
        sid = srv.add_scene(fake_scene())
        ids = [srv.submit(sid, cam(64, 64), image=image()) for _ in range(10)]
        infos = [srv.wait(i, timeout=10)[0] for i in ids]
        assert all(i["state"] == capi.DGS_REQ_DONE for i in infos)
        starts = [i["t_start"] for i in infos]
        ends = [i["t_done"] for i in infos]
        assert starts == sorted(starts)
        # one slot: a frame starts only after the previous one finished
        for a, b in zip(ends[:-1], starts[1:]):
            assert b >= a - 1e-4
        assert srv.stats()["completed"] == 10


def test_slots_run_frames_concurrently():
    def span(slots):
        with sim_server(slots=slots, fixed=0.02) as srv:
            sid = srv.add_scene(fake_scene())
            t0 = time.perf_counter()
            ids = [srv.submit(sid, cam(64, 64), image=image()) for _ in range(16)]
            for i in ids:
                srv.wait(i, timeout=10)
            return time.perf_counter() - t0
    serial, parallel = span(1), span(4)
    assert serial > 0.3
    assert parallel < serial / 2.5


def test_capacity_overflow_is_retried_and_learned():
    # 1080p at 1 key per pixel: 2.07M keys, above the 1M default capacity
    with sim_server(slots=1, keys_per_px=1.0) as srv:
        sid = srv.add_scene(fake_scene(n_cells=1000))
        a = srv.wait(srv.submit(sid, cam(1920, 1080), image=image()), timeout=10)[0]
        b = srv.wait(srv.submit(sid, cam(1920, 1080), image=image()), timeout=10)[0]
        assert a["state"] == capi.DGS_REQ_DONE and a["attempts"] == 2 and a["num_keys"] == 1920 * 1080
        assert b["state"] == capi.DGS_REQ_DONE and b["attempts"] == 1
        st = srv.stats()
        assert st["retries"] == 1
        # keys capacity was grown to the reported count plus slack
        keys = 1920 * 1080
        assert st["workspace_bytes"] >= bytes_for(0, 0, keys, 0)


def test_graph_capture_once_per_shape_and_slot():
    with sim_server(slots=1) as srv:
        sid = srv.add_scene(fake_scene())
        infos = [srv.wait(srv.submit(sid, cam(w, 64), image=image()), timeout=10)[0]
                 for w in (128, 64, 128, 64, 64, 256, 64)]
        # the 256-wide frame grows the tile workspace: captured frames of the
        # slot go stale and are captured again
        assert [i["graph"] for i in infos] == [2, 2, 1, 1, 1, 2, 2]
        st = srv.stats()
        assert st["graph_captures"] == 4 and st["graph_replays"] == 3
    with sim_server(slots=1, graphs=False) as srv:
        sid = srv.add_scene(fake_scene())
        assert srv.wait(srv.submit(sid, cam(64, 64), image=image()), timeout=10)[0]["graph"] == 0


def test_memory_budget_limits_concurrency_and_releases_idle_workspace():
    # one 1080p frame of this scene needs about 37 MB of workspace; the budget
    # holds one such frame, not two
    N, K = 100_000, 10
    tiles = 120 * 68
    need = bytes_for(int(N * 1.25), int(N * K * 1.25), max(8 * N, 1 << 20), tiles)
    with sim_server(slots=4, budget=int(need * 1.5), fixed=0.01, keys_per_px=0.1) as srv:
        sid = srv.add_scene(fake_scene(N, K))
        small = srv.add_scene(fake_scene(100, 1))
        ids = [srv.submit(sid, cam(1920, 1080), image=image()) for _ in range(6)]
        infos = [srv.wait(i, timeout=20)[0] for i in ids]
        assert all(i["state"] == capi.DGS_REQ_DONE for i in infos)
        # frames of the big scene never overlap
        iv = sorted((i["t_start"], i["t_done"]) for i in infos)
        for (s0, e0), (s1, e1) in zip(iv[:-1], iv[1:]):
            assert s1 >= e0 - 1e-3
        st = srv.stats()
        assert st["peak_workspace_bytes"] <= int(need * 1.5)
        # a small request may still run beside the big scene's slot
        assert srv.wait(srv.submit(small, cam(64, 64), image=image()), timeout=10)[0]["state"] == capi.DGS_REQ_DONE


def test_idle_slots_give_back_workspace_for_the_head_request():
    N, K = 100_000, 10
    tiles = 120 * 68
    need_a = bytes_for(int(N * 1.25), int(N * K * 1.25), 1 << 20, tiles)
    need_b = bytes_for(int(N // 2 * 1.25), int(N // 2 * K * 1.25), 1 << 20, tiles)
    budget = int(need_a * 1.3)
    assert 2 * need_b <= budget < need_a + need_b
    with sim_server(slots=4, budget=budget, fixed=0.05) as srv:
        a = srv.add_scene(fake_scene(N, K))
        b = srv.add_scene(fake_scene(N // 2, K))
        # two frames of scene b run side by side in two slots ...
        r0 = srv.submit(b, cam(1920, 1080), image=image())
        r1 = srv.submit(b, cam(1920, 1080), image=image())
        i0, i1 = srv.wait(r0, timeout=10)[0], srv.wait(r1, timeout=10)[0]
        assert i0["slot"] != i1["slot"] and i1["t_start"] < i0["t_done"]
        # ... then scene a needs one of them to give its workspace back
        info = srv.wait(srv.submit(a, cam(1920, 1080), image=image()), timeout=10)[0]
        assert info["state"] == capi.DGS_REQ_DONE
        st = srv.stats()
        assert st["releases"] == 1
        assert st["peak_workspace_bytes"] <= budget


def test_request_larger_than_budget_fails_with_oom_and_others_proceed():
    with sim_server(slots=2, budget=10_000_000) as srv:
        big = srv.add_scene(fake_scene(1_000_000, 10))
        small = srv.add_scene(fake_scene(100, 2))
        r_big = srv.submit(big, cam(1920, 1080), image=image())
        r_small = srv.submit(small, cam(64, 64), image=image())
        ib = srv.wait(r_big, timeout=10)[0]
        assert ib["state"] == capi.DGS_REQ_FAILED and ib["result"] == capi.DGS_ERR_OOM
        assert srv.wait(r_small, timeout=10)[0]["state"] == capi.DGS_REQ_DONE
        assert "budget" in srv.last_error()


def test_cancel_queued_request_only():
    with sim_server(slots=1, fixed=0.2) as srv:
        sid = srv.add_scene(fake_scene())
        r0 = srv.submit(sid, cam(64, 64), image=image())
        r1 = srv.submit(sid, cam(64, 64), image=image())
        time.sleep(0.05)
        assert srv.query(r0)["state"] == capi.DGS_REQ_RUNNING
        assert not srv.cancel(r0)
        assert srv.cancel(r1)
        assert srv.wait(r1, timeout=1)[0]["state"] == capi.DGS_REQ_CANCELLED
        assert srv.wait(r0, timeout=5)[0]["state"] == capi.DGS_REQ_DONE
        assert srv.stats()["cancelled"] == 1


def test_invalid_submissions_are_rejected_at_submit():
    with sim_server() as srv:
        sid = srv.add_scene(fake_scene())
        nocells = srv.add_scene(fake_scene(cells=False))
        with pytest.raises(capi.DgsError, match="unknown scene"):
            srv.submit(sid + 5, cam(64, 64), image=image())
        bad = cam(64, 64)
        bad["fx"] = float("nan")
        with pytest.raises(capi.DgsError, match="focal"):
            srv.submit(sid, bad, image=image())
        with pytest.raises(capi.DgsError, match="color buffer"):
            srv.submit(sid, cam(64, 64), image=capi.dgs_image(None, None, None, None))
        with pytest.raises(capi.DgsError, match="cell arrays"):
            srv.submit(nocells, cam(64, 64), image=image())
        # the same scene renders in alpha mode
        r = srv.submit(nocells, cam(64, 64), image=image(), mode="alpha")
        assert srv.wait(r, timeout=5)[0]["state"] == capi.DGS_REQ_DONE
        # a scene without Gaussian arrays is refused
        s = fake_scene()
        s.means = None
        with pytest.raises(capi.DgsError):
            srv.add_scene(s)
        # unknown request ids
        with pytest.raises(capi.DgsError):
            srv.wait(10_000, timeout=0.01)
        assert not srv.cancel(10_000)


def test_wait_times_out_on_a_running_request():
    with sim_server(slots=1, fixed=0.3) as srv:
        sid = srv.add_scene(fake_scene())
        r = srv.submit(sid, cam(64, 64), image=image())
        with pytest.raises(TimeoutError):
            srv.wait(r, timeout=0.01)
        assert srv.wait(r, timeout=5)[0]["state"] == capi.DGS_REQ_DONE


def test_destroy_cancels_queued_work_without_hanging():
    srv = sim_server(slots=1, fixed=0.05)
    sid = srv.add_scene(fake_scene())
    for _ in range(20):
        srv.submit(sid, cam(64, 64), image=image())
    t0 = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t0 < 1.0


def test_concurrent_submitters():
    with sim_server(slots=4, fixed=0.001) as srv:
        sid = srv.add_scene(fake_scene())
        out = []
        lock = threading.Lock()

        def worker():
            for _ in range(25):
                r = srv.submit(sid, cam(64, 48), image=image())
                with lock:
                    out.append(r)

        ths = [threading.Thread(target=worker) for _ in range(4)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        assert len(set(out)) == 100
        assert all(srv.wait(r, timeout=10)[0]["state"] == capi.DGS_REQ_DONE for r in out)
        assert srv.stats()["completed"] == 100


def test_poisson_load_driver_reports_latency_percentiles():
    with sim_server(slots=2, fixed=0.002) as srv:
        ids = [srv.add_scene(fake_scene())]
        cams = {0: {(64, 48): [cam(64, 48)], (128, 96): [cam(128, 96)]}}
        sched = poisson_schedule(200.0, 0.5, 1, cams, seed=5)
        assert 50 < len(sched) < 160
        res = run_load(srv, ids, sched, 200.0)
        s = res.summary()
        assert s["requests"] == len(sched) and s["failed"] == 0
        assert 2.0 <= s["p50_ms"] <= s["p99_ms"] < 100.0
        # the same seed gives the same stream
        assert [x[1] for x in poisson_schedule(200.0, 0.5, 1, cams, seed=5)] == [x[1] for x in sched]
        assert np.isclose(sched[0][0], poisson_schedule(200.0, 0.5, 1, cams, seed=5)[0][0])
