"""Workload for hardware-counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE).

Renders frames of the 1M-Gaussian clustered scene's 1920x1080 orbit in both
modes, then runs one elementwise copy kernel of known size (reads and writes
`--copy-mib` MiB each), so that per-dispatch counter values of the renderer's
kernels can be scaled by what the same counters read for a copy whose bytes
are known.

    python -m paper_2508_03180_amd.traffic --frames 6
    python -m paper_2508_03180_amd.traffic --frames 4 --modes duplex --backward
"""
from __future__ import annotations

import argparse
import sys


def main(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--frames", type=int, default=6)
    p.add_argument("--copy-mib", type=int, default=1024)
    p.add_argument("--modes", default="duplex,alpha")
    p.add_argument("--backward", action="store_true", help="also run the Duplex backward after each frame")
    a = p.parse_args(argv)
    import torch

    from . import scenes
    from .renderer import DeviceScene, Renderer

    assert torch.cuda.is_available(), "needs a HIP device"
    scene = scenes.make_mid_scene(1)
    cams = scenes.orbit_cameras(60, 1920, 1080)
    r = Renderer(0)
    ds = DeviceScene.from_numpy(scene, "cuda:0")
    out = r.alloc_image(cams[0])
    g = torch.randn((3, 1080, 1920), device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    for mode in a.modes.split(","):
        for i in range(a.frames):
            cam = cams[(10 * i) % 60]
            if a.backward and mode == "duplex":
                out = r.render(ds, cam, out=out, mode=mode, save=True)
                r.render_backward(ds, out["frame"], g)
                out.pop("frame").release()
            else:
                r.render(ds, cam, out=out, mode=mode)
        print(f"rendered {a.frames} {mode} frames" + (" with backward" if a.backward else ""), flush=True)
    n = a.copy_mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)  # reads and writes n * 4 bytes
    torch.cuda.synchronize()
    print(f"copy kernel: {n * 4} bytes read, {n * 4} bytes written", flush=True)
    r.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
