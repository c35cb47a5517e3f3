"""Writes tests/golden/clipped_energy.json: the oracle's clipped-energy
diagnostic (oracle/diagnostics.py) on the synthetic workloads -- the share
of the members' alpha mass that falls on tiles outside their cell's
footprint, which the tile lists cut away (the cell footprint reading of the
paper's Sec. IV-B, whose containment constraints of eqs. `scaffold_offset`
and `scale_res` the synthetic scenes do not enforce).

Calls only the oracle and the seeded scene generators.  Run from the
repository root:

    python tests/golden/make_clipped_energy.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import diagnostics  # noqa: E402
from paper_2508_03180_amd import scenes  # noqa: E402

SAMPLE = 20000


def entry(scene, cam, name, sample):
    d = diagnostics.clipped_alpha_mass(scene, cam, sample=sample, seed=0)
    d["workload"] = name
    d["sampled"] = sample is not None and d["members"] == sample
    print(name, round(d["fraction"], 5), d["members"], flush=True)
    return d


def main():
    out = []
    out.append(entry(scenes.make_tiny_scene(0), scenes.tiny_camera(), "tiny scene (2,000 cells x 8), 256x256", None))
    mid = scenes.make_mid_scene(1)
    cams = scenes.orbit_cameras(60, 1920, 1080)
    for i in (0, 30):
        out.append(entry(mid, cams[i], f"mid scene (100,000 cells x 10), 1920x1080 orbit frame {i}", SAMPLE))
    del mid
    large = scenes.make_large_scene(2)
    for (w, h) in ((1280, 720), (1920, 1080)):
        allc = scenes.large_scene_cameras(2, w, h, n_near=20, n_far=20)
        for kind, cam in (("near camera 0", allc[0]), ("far camera 0", allc[20])):
            out.append(entry(large, cam, f"large scene (600,000 cells x 10), {w}x{h} {kind}", SAMPLE))
    doc = {
        "what": "share of the members' alpha mass (min(alpha_max, sigma G') over each member's 3-sigma box, "
                "where it passes alpha_min, before transmittance) on tiles outside the member's cell footprint",
        "source": "oracle/diagnostics.py via tests/golden/make_clipped_energy.py",
        "sample": f"a seeded random sample of {SAMPLE} listed members where a workload has more",
        "results": out,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "clipped_energy.json"), "w") as f:
        json.dump(doc, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
