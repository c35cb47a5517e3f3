"""A caller captures a frame into a HIP graph itself.

The frame forks its member projection onto the context's second stream and
joins it back, so the capture must take both streams' work; the replays,
with other frames rendered eagerly and synchronisations between them, must
each give the eager frame's bits.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2508_03180_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["duplex", "alpha"])
def test_caller_captured_frame_replays_exactly(mode):
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer
    s = scenes.make_tiny_scene(0)
    cams = [scenes.tiny_camera(), scenes.orbit_cameras(12, 256, 256, radius=3.0)[4]]
    side = torch.cuda.Stream()
    r = Renderer(0, stream=side)
    try:
        ds = DeviceScene.from_numpy(s, "cuda:0")
        with torch.cuda.stream(side):
            ref = {k: v.clone() for k, v in r.render(ds, cams[0], mode=mode).items()}  # sizes the workspace
            other = {k: v.clone() for k, v in r.render(ds, cams[1], mode=mode).items()}
            out = r.alloc_image(cams[0])
            side.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                r.render(ds, cams[0], out=out, mode=mode, check=False)  # enqueue only
        for rep in range(3):
            for v in out.values():
                v.fill_(0)
            g.replay()
            torch.cuda.synchronize()
            for k in ("color", "D", "T", "last"):
                assert torch.equal(out[k], ref[k]), (mode, rep, k)
            with torch.cuda.stream(side):  # eager work between replays
                o2 = r.render(ds, cams[1], mode=mode)
            torch.cuda.synchronize()
            assert torch.equal(o2["color"], other["color"])
        assert _capi.dgs_sync(r.ctx) == 0
    finally:
        r.close()
