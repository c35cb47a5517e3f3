"""Both ways to the lists' depth order -- a depth sort of the primitives
before the key emission, or a sort of each tile's run after the tile sort --
give the oracle's (tile, depth bits, id) lists bit for bit, and the same
images and saved frames (Sec. IV-B)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_03180_amd import _capi as capi
from paper_2508_03180_amd import scenes

pytestmark = pytest.mark.gpu

ORDERS = {"per_tile": capi.DGS_LIST_ORDER_PER_TILE, "global": capi.DGS_LIST_ORDER_GLOBAL,
          "auto": capi.DGS_LIST_ORDER_AUTO}


@pytest.fixture(scope="module")
def rs():
    from paper_2508_03180_amd.renderer import Renderer
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    out = {}
    for name, v in ORDERS.items():
        r = Renderer(0)
        assert capi.dgs_set_list_order(r.ctx, v) == capi.DGS_OK
        out[name] = r
    yield out
    for r in out.values():
        r.close()


def crowded_tile_scene(n=6000, seed=5):
    """n small cells in front of a 32 x 16 image (two tiles), most of them
    covering tile 0, half of them at one depth: runs longer than a
    workgroup sorts in registers (2,048 entries), with thousands of exact
    depth ties."""
    rng = np.random.default_rng(seed)
    s = scenes.make_tiny_scene(seed, n_cells=n, K=2)
    z = np.where(rng.random(n) < 0.5, 3.0, rng.uniform(2.0, 4.0, n)).astype(np.float32)
    x = rng.uniform(-0.15, 0.05, n).astype(np.float32) * z / 1.0
    y = rng.uniform(-0.1, 0.1, n).astype(np.float32) * z / 1.0
    s["cell_pos"] = np.stack([x, y, z], 1).astype(np.float32)
    s["cell_scale"] = np.full((n, 3), 0.01, np.float32)
    s["means"] = np.repeat(s["cell_pos"], 2, 0)
    cam = dict(viewmat=np.eye(4, dtype=np.float32), fx=40.0, fy=40.0, cx=16.0, cy=8.0, width=32, height=16,
               z_near=0.2)
    return s, cam


def cases():
    return ["tiny", "mid0", "mid45", "alpha_tiny", "alpha_mid0", "crowded"]


def scene_for(case):
    if case in ("tiny", "alpha_tiny"):
        return scenes.make_tiny_scene(0), scenes.tiny_camera(), ("alpha" if case == "alpha_tiny" else "duplex")
    if case == "crowded":
        s, cam = crowded_tile_scene()
        return s, cam, "duplex"
    frame = int(case.split("mid")[1])
    mode = "alpha" if case.startswith("alpha") else "duplex"
    return scenes.make_mid_scene(1), scenes.orbit_cameras(60, 1920, 1080)[frame], mode


@pytest.mark.parametrize("case", cases())
def test_both_orders_give_the_oracle_lists(rs, case):
    from paper_2508_03180_amd.renderer import DeviceScene
    s, cam, mode = scene_for(case)
    ds = DeviceScene.from_numpy(s, "cuda:0")
    W, H = cam["width"], cam["height"]
    tiles = ((W + 15) // 16) * ((H + 15) // 16)
    d = oracle.cells_discrete(s, cam) if mode == "duplex" else oracle.gauss_discrete(s, cam)
    ids, otiles, oranges = oracle.build_lists(d["visible"], d["depth_bits"], d["rect"], W, H)
    want_keys = (otiles.astype(np.uint64) << np.uint64(32)) | d["depth_bits"][ids].astype(np.uint64)
    images, passes = {}, {}
    for name, r in rs.items():
        out = r.render(ds, cam, mode=mode)
        keys, vals, ranges = r.read_lists(tiles)
        torch.cuda.synchronize()
        assert keys.numel() == len(ids), (name, case)
        np.testing.assert_array_equal(vals.cpu().numpy(), ids, err_msg=f"{name} {case}")
        np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint64), want_keys, err_msg=f"{name} {case}")
        np.testing.assert_array_equal(ranges.cpu().numpy(), oranges, err_msg=f"{name} {case}")
        images[name] = {k: v.clone() for k, v in out.items()}
        passes[name] = r.stats()["sort_passes"]
    # the per-tile order runs no depth sort (four 8-bit passes over the depth bits)
    assert passes["per_tile"] == passes["global"] - 4, passes
    # the default takes one of the two (per-Gaussian lists: always global)
    assert passes["auto"] in (passes["per_tile"], passes["global"]), (case, passes)
    if mode == "alpha":
        assert passes["auto"] == passes["global"], (case, passes)
    if case == "crowded":
        assert int((oranges[:, 1] - oranges[:, 0]).max()) > 4096  # chunks merged over two rounds
    for k in ("color", "D", "T", "last"):
        assert torch.equal(images["per_tile"][k], images["global"][k]), (case, k)
        assert torch.equal(images["auto"][k], images["global"][k]), (case, k)


def test_saved_frames_and_gradients_agree(rs):
    """The per-tile order also fills the saved frame's lists: the backward
    of a frame saved either way gives the same gradients (up to the order of
    the float atomics)."""
    from paper_2508_03180_amd.renderer import DeviceScene
    s = scenes.make_tiny_scene(2)
    cam = scenes.tiny_camera()
    ds = DeviceScene.from_numpy(s, "cuda:0")
    g = torch.randn((3, cam["height"], cam["width"]), device="cuda", generator=torch.Generator("cuda").manual_seed(1))
    grads = {}
    for name, r in rs.items():
        out = r.render(ds, cam, save=True)
        grads[name] = r.render_backward(ds, out["frame"], g)
        out["frame"].release()
    torch.cuda.synchronize()
    for k in grads["global"]:
        b = grads["global"][k].double()
        for name in ("per_tile", "auto"):
            a = grads[name][k].double()
            assert float((a - b).norm()) <= 1e-5 * max(float(b.norm()), 1e-30), (name, k)


def tile_passes(cam):
    tiles = ((cam["width"] + 15) // 16) * ((cam["height"] + 15) // 16)
    return (max(1, (tiles - 1).bit_length()) + 7) // 8


def test_default_order_follows_the_last_frame():
    """DGS_LIST_ORDER_AUTO: per tile when the context's last cell frame had
    at most 8 keys per cell, at most 1024 keys per tile
    and at most a twentieth of its keys in runs of more than 4096 entries, else
    global; before any frame, by the key capacity (at most 256 keys per
    tile).  The frames are synchronised, so each choice sees the frame
    before it."""
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer
    tiny, tcam, _ = scene_for("tiny")
    mid, mcam, _ = scene_for("mid0")
    crowd, ccam, _ = scene_for("crowded")
    dt, dm, dc = (DeviceScene.from_numpy(x, "cuda:0") for x in (tiny, mid, crowd))
    r = Renderer(0)
    try:
        steps = [(dt, tcam, False),  # capacity 2^20 keys over 256 tiles
                 (dm, mcam, True),   # tiny: 22 keys per tile
                 (dc, ccam, True),   # 1080p orbit frame: 64 keys per tile
                 (dm, mcam, False),  # crowded: 3,958 keys per tile, 69% in a run over 4096
                 (dm, mcam, True)]
        images = []
        for i, (ds, cam, per_tile) in enumerate(steps):
            out = r.render(ds, cam)
            torch.cuda.synchronize()
            want = tile_passes(cam) + (0 if per_tile else 4)
            assert r.stats()["sort_passes"] == want, (i, r.stats()["sort_passes"], want)
            if ds is dm:
                images.append({k: v.clone() for k, v in out.items()})
        for k in ("color", "D", "T", "last"):
            assert torch.equal(images[1][k], images[2][k]), k
    finally:
        r.close()


def test_invalid_list_order(rs):
    r = rs["global"]
    assert capi.dgs_set_list_order(r.ctx, 3) == capi.DGS_ERR_INVALID_ARG
    assert capi.dgs_set_list_order(r.ctx, -1) == capi.DGS_ERR_INVALID_ARG
