"""Frames in flight: several renderers (contexts on their own streams) render
different frames of one resident scene at the same time; every frame is
bit-identical to the same frame rendered alone, with the in-frame second
stream on or off."""
import numpy as np
import pytest
import torch

from paper_2508_03180_amd import _capi as capi
from paper_2508_03180_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["duplex", "alpha"])
@pytest.mark.parametrize("scene_kind", ["tiny", "mid"])
def test_concurrent_renderers_match_frames_rendered_alone(mode, scene_kind):
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer, camera_struct, opts_struct
    if scene_kind == "tiny":
        s = scenes.make_tiny_scene(0)
        cams = scenes.orbit_cameras(12, 256, 256, radius=3.0)
    else:
        s = scenes.make_mid_scene(1)
        cams = scenes.orbit_cameras(60, 1920, 1080)[::10]
    ds = DeviceScene.from_numpy(s, "cuda:0")
    alone = Renderer(0)
    want = [alone.render(ds, c, mode=mode)["color"].clone() for c in cams]
    torch.cuda.synchronize()
    # three renderers without in-frame overlap and one with it
    rs = [Renderer(0, stream=torch.cuda.Stream(), overlap=(i == 3)) for i in range(4)]
    try:
        for r in rs:  # size every workspace
            for c in cams:
                r.render(ds, c, mode=mode)
        torch.cuda.synchronize()
        L = capi.lib()
        sc = ds.struct()
        op = opts_struct(mode=mode)
        outs = [[r.alloc_image(cams[0]) for _ in cams] for r in rs]
        # every renderer renders every frame, the renderers interleaved, all
        # enqueued before any is waited for
        for i, c in enumerate(cams):
            cs = camera_struct(c)
            for j, r in enumerate(rs):
                o = outs[j][i]
                im = capi.dgs_image(o["color"].data_ptr(), o["D"].data_ptr(), o["T"].data_ptr(),
                                    o["last"].data_ptr())
                assert L.dgs_render(r.ctx, sc, cs, op, im, None) == 0
        torch.cuda.synchronize()
        for j, r in enumerate(rs):
            assert capi.dgs_sync(r.ctx) == 0
            for i in range(len(cams)):
                assert torch.equal(outs[j][i]["color"], want[i]), (mode, scene_kind, j, i)
    finally:
        for r in rs:
            r.close()
        alone.close()


def test_overlap_switch_leaves_frames_unchanged():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer
    s = scenes.make_tiny_scene(1)
    cam = scenes.tiny_camera()
    ds = DeviceScene.from_numpy(s, "cuda:0")
    a, b = Renderer(0), Renderer(0, overlap=False)
    try:
        for k in ("color", "D", "T", "last"):
            x = a.render(ds, cam)[k]
            y = b.render(ds, cam)[k]
            torch.cuda.synchronize()
            assert torch.equal(x, y), k
        assert capi.dgs_set_overlap(b.ctx, True) == capi.DGS_OK
        assert torch.equal(b.render(ds, cam)["color"], a.render(ds, cam)["color"])
    finally:
        a.close()
        b.close()
