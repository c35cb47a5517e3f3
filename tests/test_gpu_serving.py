"""Serving runtime on the GPU: every request served in a mixed load (several
scenes, sizes, modes and options, frames in flight on several streams,
captured graphs replayed with new cameras) is bit-identical to the same
request rendered alone with dgs_render, whose parity with the oracle the
parity tests establish."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2508_03180_amd import _capi as capi
from paper_2508_03180_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer
    tiny = scenes.make_tiny_scene(0)
    mid = scenes.make_mid_scene(40, n_cells=20_000)
    ds = [DeviceScene.from_numpy(tiny, "cuda:0"), DeviceScene.from_numpy(mid, "cuda:0")]
    r = Renderer(0)
    yield ds, r
    r.close()


def cameras(scene_idx, w, h, n=6):
    if scene_idx == 0:
        base = scenes.orbit_cameras(n, w, h, radius=3.0, elevation_deg=20.0, step_deg=60.0 / n)
    else:
        base = scenes.orbit_cameras(n, w, h)
    return base


OPTS = [dict(), dict(mode="alpha"), dict(bg=(0.2, 0.4, 0.6)), dict(v_one=True), dict(no_et=True)]
SIZES = [(256, 256), (333, 197), (640, 480), (1280, 720)]


def mixed_requests(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        s = int(rng.integers(2))
        w, h = SIZES[int(rng.integers(len(SIZES)))]
        cam = cameras(s, w, h)[int(rng.integers(6))]
        o = OPTS[int(rng.integers(len(OPTS)))]
        out.append((s, cam, o))
    return out


def alone(r, ds, s, cam, o):
    return r.render(ds[s], cam, **o)["color"]


def serve_and_compare(dev, server_kw, reqs):
    from paper_2508_03180_amd.serving import Server
    ds, r = dev
    with Server(0, **server_kw) as srv:
        ids = [srv.add_scene(d) for d in ds]
        rids = [srv.submit(ids[s], cam, **o) for (s, cam, o) in reqs]
        results = [srv.wait(i, timeout=60) for i in rids]
        stats = srv.stats()
    torch.cuda.synchronize()
    for (info, img), (s, cam, o) in zip(results, reqs):
        assert info["state"] == capi.DGS_REQ_DONE, (info, s, cam["width"], o)
        ref = alone(r, ds, s, cam, o)
        assert torch.equal(img, ref), (s, cam["width"], cam["height"], o)
    return results, stats


def test_mixed_load_is_bit_identical_to_rendering_alone(dev):
    reqs = mixed_requests(1, 48)
    results, st = serve_and_compare(dev, dict(num_slots=4, use_graphs=True), reqs)
    assert st["graph_captures"] >= 1 and st["graph_replays"] >= 1
    assert st["completed"] == len(reqs)
    assert max(i["slot"] for i, _ in results) >= 1  # more than one slot took work


def test_mixed_load_without_graphs(dev):
    reqs = mixed_requests(2, 16)
    _, st = serve_and_compare(dev, dict(num_slots=3, use_graphs=False), reqs)
    assert st["graph_captures"] == 0


def test_capacity_overflow_is_retried_on_the_device(dev):
    """Large cells at 1080p produce more keys than the first estimate; the
    server grows the slot and runs the frame again."""
    from paper_2508_03180_amd.renderer import DeviceScene
    from paper_2508_03180_amd.serving import Server
    _, r = dev
    s = scenes.make_tiny_scene(0)
    s["cell_scale"] = (s["cell_scale"] * 10.0).astype(np.float32)
    big = DeviceScene.from_numpy(s, "cuda:0")
    cam = scenes.orbit_cameras(1, 1920, 1080)[0]
    with Server(0, num_slots=2) as srv:
        sid = srv.add_scene(big)
        a = srv.wait(srv.submit(sid, cam), timeout=60)
        b = srv.wait(srv.submit(sid, cam), timeout=60)
        st = srv.stats()
    assert a[0]["state"] == capi.DGS_REQ_DONE and a[0]["attempts"] == 2 and a[0]["num_keys"] > (1 << 20)
    assert b[0]["attempts"] == 1 and st["retries"] == 1
    ref = r.render(big, cam)["color"]
    assert torch.equal(a[1], ref) and torch.equal(b[1], ref)


def test_memory_budget_on_the_device(dev):
    """A budget that holds about one workspace: frames wait for memory instead
    of running side by side, and results stay identical."""
    reqs = [(i % 2, cameras(i % 2, 1280, 720)[i % 6], {}) for i in range(8)]
    results, st = serve_and_compare(dev, dict(num_slots=4, use_graphs=True, memory_budget=48 << 20), reqs)
    assert st["peak_workspace_bytes"] <= 48 << 20


def test_full_size_scenes_and_4k_in_the_mix(dev):
    """The serving benchmark's full-size scenes -- the 1M-Gaussian clustered
    scene and the 6M-Gaussian large scene -- with 1920x1080 and 3840x2160
    requests among small ones, several frames in flight with graph replay:
    every result is bit-identical to the same request rendered alone."""
    from paper_2508_03180_amd.renderer import DeviceScene
    from paper_2508_03180_amd.serving import Server
    _, r = dev
    big = [DeviceScene.from_numpy(scenes.make_mid_scene(41), "cuda:0"),
           DeviceScene.from_numpy(scenes.make_large_scene(43), "cuda:0")]
    rng = np.random.default_rng(9)
    reqs = []
    for i in range(14):
        s = i % 2
        w, h = [(640, 480), (1920, 1080), (3840, 2160)][int(rng.integers(3))] if i > 1 else (3840, 2160)
        cams = scenes.orbit_cameras(12, w, h, step_deg=30.0) if s == 0 else \
            scenes.aerial_orbit_cameras(12, w, h, step_deg=30.0)
        reqs.append((s, cams[int(rng.integers(12))], OPTS[int(rng.integers(2))]))
    with Server(0, num_slots=4, use_graphs=True) as srv:
        ids = [srv.add_scene(d) for d in big]
        rids = [srv.submit(ids[s], cam, **o) for (s, cam, o) in reqs]
        results = [srv.wait(i, timeout=120) for i in rids]
        st = srv.stats()
        err = srv.last_error()
    torch.cuda.synchronize()
    for (info, img), (s, cam, o) in zip(results, reqs):
        assert info["state"] == capi.DGS_REQ_DONE, (info, err, st, s, cam["width"], o)
    assert st["completed"] == len(reqs) and max(i["slot"] for i, _ in results) >= 1
    assert any(cam["width"] == 3840 for _, cam, _ in reqs)
    for (info, img), (s, cam, o) in zip(results, reqs):
        assert torch.equal(img, r.render(big[s], cam, **o)["color"]), (s, cam["width"], o)
