"""Pins of the clipped-energy diagnostic (oracle/diagnostics.py) against
closed forms (CPU only)."""
import numpy as np
import pytest

from oracle import diagnostics
from paper_2508_03180_amd import scenes
from test_oracle_pins import axis_camera, manual_scene


def one_member(cell_u, member_u, member_scale, cell_scale=0.01, W=32, H=16, f=200.0, z=4.0):
    """One cell and one member on the image's middle row; screen positions
    given in pixels (u = f x / z + W / 2)."""
    cam = axis_camera(W, H, f)
    x_cell = (cell_u - W / 2) * z / f
    x_mem = (member_u - W / 2) * z / f
    sc = manual_scene([dict(pos=[x_cell, 0.0, z], scale=[cell_scale] * 3,
                            members=[dict(mean=[x_mem, 0.0, z], scale=[member_scale] * 3, sigma=0.9,
                                          rgb=[1, 1, 1])])], K=1)
    return sc, cam


def test_member_on_a_tile_edge_loses_exactly_half():
    """An isotropic member centred on the edge between tile columns 0 and 1
    (u = 16, box pixels 7..24) whose cell's footprint lies in column 0: the
    pixel grid is mirror-symmetric about the edge, so half the mass is cut."""
    sc, cam = one_member(cell_u=8.0, member_u=16.0, member_scale=0.06)
    d = diagnostics.clipped_alpha_mass(sc, cam)
    assert d["members"] == 1 and d["members_clipped"] == 1
    assert d["fraction"] == pytest.approx(0.5, abs=1e-12)


def test_member_inside_a_footprint_covering_the_image_loses_nothing():
    sc, cam = one_member(cell_u=16.0, member_u=16.0, member_scale=0.06, cell_scale=5.0)
    d = diagnostics.clipped_alpha_mass(sc, cam)
    assert d["fraction"] == 0.0 and d["members_clipped"] == 0 and d["total_mass"] > 0


def test_member_far_from_its_cell_loses_everything():
    """Cell footprint in tile column 0, member box (u = 28, screen sigma 1
    px: pixels 25..31) entirely in column 1."""
    sc, cam = one_member(cell_u=6.0, member_u=28.0, member_scale=0.02)
    d = diagnostics.clipped_alpha_mass(sc, cam)
    assert d["fraction"] == 1.0


def test_sampling_every_member_equals_the_full_sum():
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    full = diagnostics.clipped_alpha_mass(s, cam)
    samp = diagnostics.clipped_alpha_mass(s, cam, sample=10 ** 9)
    assert samp["fraction"] == full["fraction"] and samp["members"] == full["members"]
    part = diagnostics.clipped_alpha_mass(s, cam, sample=2000, seed=3)
    assert part["members"] == 2000 and 0.0 <= part["fraction"] <= 1.0


def test_ragged_cells_equal_the_padded_scene():
    """Padding members are invalid (sigma 0): they hold no mass and move no
    cell, so the CSR scene and its padded copy give the same diagnostic."""
    s = scenes.make_ragged_scene(4, n_cells=300)
    cam = scenes.tiny_camera()
    a = diagnostics.clipped_alpha_mass(s, cam)
    b = diagnostics.clipped_alpha_mass(scenes.pad_to_fixed_k(s), cam)
    assert a["members"] == b["members"] and a["fraction"] == pytest.approx(b["fraction"], rel=1e-12)
    assert np.array_equal(diagnostics.member_cells(s), np.repeat(np.arange(300), np.diff(s["cell_offsets"])))


def test_stored_diagnostic_matches_the_oracle():
    """tests/golden/clipped_energy.json was written by
    tests/golden/make_clipped_energy.py from the oracle; its tiny-scene entry
    (every member, no sampling) is recomputed here."""
    import json
    import os
    doc = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "clipped_energy.json")))
    tiny = doc["results"][0]
    assert tiny["workload"].startswith("tiny scene") and not tiny["sampled"]
    d = diagnostics.clipped_alpha_mass(scenes.make_tiny_scene(0), scenes.tiny_camera())
    assert d["members"] == tiny["members"] and d["fraction"] == pytest.approx(tiny["fraction"], rel=1e-12)
    assert all(0.0 <= r["fraction"] < 0.1 for r in doc["results"])
