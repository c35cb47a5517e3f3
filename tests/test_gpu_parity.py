"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Integer work (pixel rectangles, depth keys, tile counts, sorted lists, the
radix sort) must match bit for bit; pixels must be within 2e-4 max-abs per
channel of the oracle under the admissible-set rule for threshold decisions
that fall within rounding of alpha_min or eps.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2508_03180_amd import scenes

pytestmark = pytest.mark.gpu

TOL = 2e-4


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2508_03180_amd.renderer import Renderer
    r = Renderer(0)
    yield r
    r.close()


def upload(s):
    from paper_2508_03180_amd.renderer import DeviceScene
    return DeviceScene.from_numpy(s, "cuda:0")


def flat(t):
    return t.permute(1, 2, 0).reshape(-1, 3).double().cpu().numpy()


def check_image(out, ref, tol=TOL, max_unverifiable=1e-3):
    err = oracle.admissible_max_err(flat(out["color"]), ref)
    ok = np.isfinite(err)
    assert 1 - ok.mean() <= max_unverifiable, f"unverifiable {1 - ok.mean():.2e}"
    worst = float(np.nanmax(err)) if ok.any() else 0.0
    assert worst <= tol, f"max abs error {worst:.3e} at pixel {int(np.nanargmax(err))}"
    return err


def check_aux(out, ref, d_rtol=0.0):
    """D and T within the tolerance and `last` (an index) equal on every
    pixel without a marginal threshold decision."""
    exact = ref["status"] == 0
    D = out["D"].reshape(-1).double().cpu().numpy()
    T = out["T"].reshape(-1).double().cpu().numpy()
    np.testing.assert_allclose(D[exact], ref["D"][exact], rtol=d_rtol, atol=TOL)
    np.testing.assert_allclose(T[exact], ref["T"][exact], atol=TOL)
    last = out["last"].reshape(-1).cpu().numpy()
    np.testing.assert_array_equal(last[exact], ref["last"][exact])


# ------------------------------------------------------------------ sort

@pytest.mark.parametrize("n,bits", [(1, 8), (2, 40), (3071, 40), (3072, 44), (3073, 45), (100_003, 45),
                                    (1_000_000, 47), (65_537, 64), (5000, 1)])
def test_sort_pairs_matches_stable_argsort(R, n, bits):
    rng = np.random.default_rng(n + bits)
    hi = (1 << bits) if bits < 64 else None
    if hi is None:
        k = rng.integers(0, 2 ** 63 - 1, n, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, n).astype(np.uint64)
    else:
        # few distinct values so that ties (stability) matter
        k = rng.integers(0, min(hi, max(4, n // 3)), n, dtype=np.int64).astype(np.uint64)
        k = (k * np.uint64(0x9E3779B1)) & np.uint64(hi - 1)
    v = np.arange(n, dtype=np.int32)
    kt = torch.from_numpy(k.view(np.int64)).cuda()
    vt = torch.from_numpy(v).cuda()
    R.sort_pairs(kt, vt, bits)
    order = np.argsort(k, kind="stable")
    np.testing.assert_array_equal(kt.cpu().numpy().view(np.uint64), k[order])
    np.testing.assert_array_equal(vt.cpu().numpy(), v[order])


def test_sort_all_equal_keys_is_identity(R):
    n = 50_000
    kt = torch.full((n,), 0x12345678, dtype=torch.int64, device="cuda")
    vt = torch.arange(n, dtype=torch.int32, device="cuda")
    R.sort_pairs(kt, vt, 40)
    assert (vt.cpu().numpy() == np.arange(n)).all()


# ------------------------------------------------------------------ discrete layer

def _c1_scene():
    return scenes.make_mid_scene(1)


@pytest.fixture(scope="module")
def c1():
    return _c1_scene()


def _check_discrete(R, s, cam):
    ds = upload(s)
    R.render(ds, cam)
    rect, depth, nt = R.read_prims(ds.N)
    cd = oracle.cells_discrete(s, cam)
    np.testing.assert_array_equal(rect.cpu().numpy(), cd["rect"])
    np.testing.assert_array_equal(depth.cpu().numpy().view(np.uint32), cd["depth_bits"])
    np.testing.assert_array_equal(nt.cpu().numpy(), cd["ntiles"])
    keys, vals, ranges = R.read_lists(((cam["width"] + 15) // 16) * ((cam["height"] + 15) // 16))
    ids, tiles, oranges = oracle.build_lists(cd["visible"], cd["depth_bits"], cd["rect"], cam["width"], cam["height"])
    assert keys.numel() == len(ids)
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal((keys.cpu().numpy().view(np.uint64) >> np.uint64(32)).astype(np.int32), tiles)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)
    # member rectangles of projected cells
    gr = R.read_gauss_rects(ds.M).cpu().numpy()
    gd = oracle.gauss_discrete(s, cam)
    proj = np.repeat(cd["visible"].astype(bool), s["K"])
    np.testing.assert_array_equal(gr[proj], gd["rect"][proj])
    return len(ids)


def test_discrete_layer_bit_exact_tiny(R):
    n = _check_discrete(R, scenes.make_tiny_scene(0), scenes.tiny_camera())
    assert n > 1000


@pytest.mark.parametrize("frame", [0, 17, 45])
def test_discrete_layer_bit_exact_1080p(R, c1, frame):
    cam = scenes.orbit_cameras(60, 1920, 1080)[frame]
    n = _check_discrete(R, c1, cam)
    assert n > 100_000


@pytest.mark.parametrize("size,cell_mult", [((8192, 128), 30.0), ((5000, 4000), 3.0)])
def test_discrete_layer_bit_exact_wide_images(R, size, cell_mult):
    """Tile rows longer than 256 tiles (8192 px wide, cells thousands of
    pixels across) and tile ids above 2^16 (313 x 250 tiles, a 7-pass sort):
    the key emission's run-length digit counting must give the sort the
    exact histogram."""
    s = scenes.make_tiny_scene(0)
    s["cell_scale"] = (s["cell_scale"] * cell_mult).astype(np.float32)
    base = scenes.tiny_camera()
    cam = scenes.pinhole(base["viewmat"], size[0], size[1])
    n = _check_discrete(R, s, cam)
    assert n > 1_000_000


def test_gaussian_keys_bit_exact_alpha_mode(R):
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    ds = upload(s)
    R.render(ds, cam, mode="alpha")
    rect, depth, nt = R.read_prims(ds.M)
    gd = oracle.gauss_discrete(s, cam)
    np.testing.assert_array_equal(rect.cpu().numpy(), gd["rect"])
    np.testing.assert_array_equal(nt.cpu().numpy(), gd["ntiles"])
    keys, vals, ranges = R.read_lists(256)
    ids, _, oranges = oracle.build_lists(gd["visible"], gd["depth_bits"], gd["rect"], 256, 256)
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)


def _tie_scene():
    """Cells and Gaussians on three planes of constant camera depth (an
    axis-aligned camera makes their depth bits equal), the last third of
    the cells exact copies of the first third in reverse order: the sorted
    lists must break every depth tie by ascending id."""
    s = scenes.make_tiny_scene(3, n_cells=3000)
    rng = np.random.default_rng(3)
    N = s["cell_pos"].shape[0]
    s["cell_pos"][:, 2] = rng.choice(np.float32([-0.5, 0.0, 0.5]), N)
    s["means"][:, 2] = rng.choice(np.float32([-0.25, 0.25]), s["means"].shape[0])
    d = N // 3
    for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh"):
        s[k][N - d:] = s[k][:d][::-1]
    view = np.eye(4, dtype=np.float32)
    view[2, 3] = 3.0
    return s, scenes.pinhole(view, 256, 256)


def _count_ties(keys):
    k = keys.cpu().numpy().view(np.uint64)
    return int((k[1:] == k[:-1]).sum())


def test_sorted_lists_break_depth_ties_by_id(R):
    s, cam = _tie_scene()
    n = _check_discrete(R, s, cam)
    keys, _, _ = R.read_lists(256)
    assert n > 1000 and _count_ties(keys) > 1000


def test_sorted_gaussian_lists_break_depth_ties_by_id(R):
    s, cam = _tie_scene()
    ds = upload(s)
    R.render(ds, cam, mode="alpha")
    gd = oracle.gauss_discrete(s, cam)
    keys, vals, ranges = R.read_lists(256)
    ids, _, oranges = oracle.build_lists(gd["visible"], gd["depth_bits"], gd["rect"], 256, 256)
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)
    assert _count_ties(keys) > 1000


# ------------------------------------------------------------------ images

def test_tiny_scene_image_parity(R):
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    out = R.render(upload(s), cam)
    ref = oracle.render(s, cam)
    check_image(out, ref)
    check_aux(out, ref)


# The compositor splits a tile whose list has at least 32 cells (64 Gaussians
# in the per-Gaussian mode) into two half-tile work items.  Tiny scenes 1 and
# 2 hold tiles whose cell lists are one short of, exactly at and one past 32,
# and scene 2 tiles with 63 and 64 Gaussians; their pixels, lists and ranges
# are checked here.
SPLIT_LEN = {"duplex": 32, "alpha": 64}


def split_boundary_pixels(s, cam, mode):
    if mode == "duplex":
        d = oracle.cells_discrete(s, cam)
    else:
        d = oracle.gauss_discrete(s, cam)
    W, H = cam["width"], cam["height"]
    _, _, ranges = oracle.build_lists(d["visible"], d["depth_bits"], d["rect"], W, H)
    lens = ranges[:, 1] - ranges[:, 0]
    L = SPLIT_LEN[mode]
    tiles = np.nonzero((lens >= L - 1) & (lens <= L + 1))[0]
    TX = (W + 15) // 16
    mask = np.zeros((H, W), bool)
    for t in tiles:
        ty, tx = divmod(int(t), TX)
        mask[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = True
    return tiles, lens[tiles], mask.reshape(-1)


@pytest.mark.parametrize("seed,mode", [(1, "duplex"), (2, "duplex"), (2, "alpha")])
def test_tiles_at_the_split_length(R, seed, mode):
    s = scenes.make_tiny_scene(seed)
    cam = scenes.tiny_camera()
    tiles, lens, mask = split_boundary_pixels(s, cam, mode)
    L = SPLIT_LEN[mode]
    assert len(tiles) > 0 and lens.min() < L <= lens.max()
    out = R.render(upload(s), cam, mode=mode)
    keys, vals, ranges = R.read_lists(256)
    d = oracle.cells_discrete(s, cam) if mode == "duplex" else oracle.gauss_discrete(s, cam)
    ids, _, oranges = oracle.build_lists(d["visible"], d["depth_bits"], d["rect"], 256, 256)
    assert keys.numel() == len(ids)
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)
    ref = oracle.render(s, cam, mode=mode)
    err = oracle.admissible_max_err(flat(out["color"]), ref)[mask]
    assert np.isfinite(err).mean() >= 0.999
    assert np.nanmax(err) <= TOL


@pytest.mark.parametrize("flags", [dict(v_one=True), dict(no_et=True), dict(bg=(0.2, 0.4, 0.6)),
                                   dict(kappa=3.0), dict(eps=1e-2)])
def test_tiny_scene_option_parity(R, flags):
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    out = R.render(upload(s), cam, **flags)
    ref = oracle.render(s, cam, **flags)
    check_image(out, ref)
    check_aux(out, ref)


def test_tiny_scene_alpha_mode_parity(R):
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    out = R.render(upload(s), cam, mode="alpha")
    ref = oracle.render(s, cam, mode="alpha")
    check_image(out, ref)
    check_aux(out, ref)


@pytest.mark.parametrize("flags", [dict(tau=4.5), dict(tau=3.2, v_one=True), dict(tau=4.5, bg=(0.3, 0.1, 0.2)),
                                   dict(tau=3.0, kappa=3.0)])
def test_tiny_scene_lcwsr_parity(R, flags):
    """The "w/o T^cell" mode (LC-WSR cell weights): whole image against the
    oracle; no transmittance (T = 1) and the last contributing entry."""
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    out = R.render(upload(s), cam, mode="lcwsr", **flags)
    ref = oracle.render(s, cam, mode="lcwsr", **flags)
    check_image(out, ref)
    check_aux(out, ref, d_rtol=1e-5)
    assert (out["T"] == 1.0).all()


def test_lcwsr_mode_is_checked_and_has_no_backward(R):
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import opts_struct
    s = upload(scenes.make_tiny_scene(0))
    cam = scenes.tiny_camera()
    out = R.alloc_image(cam)
    assert R.render_into(s, cam, out, opts_struct(mode="lcwsr")) == _capi.DGS_ERR_INVALID_ARG
    assert R.render_into(s, cam, out, opts_struct(mode="lcwsr", tau=float("inf"))) == _capi.DGS_ERR_INVALID_ARG
    R.render(s, cam, out=out, mode="lcwsr", tau=4.0)
    with pytest.raises(_capi.DgsError, match="UNSUPPORTED"):
        R.render(s, cam, out=out, mode="lcwsr", tau=4.0, save=True)


def test_ragged_image_and_opaque_scene(R):
    """Image sides that are not multiples of 16 (partial tiles) and a scene of
    near-opaque Gaussians (early termination on most pixels)."""
    s = scenes.make_tiny_scene(3, n_cells=3000, K=6)
    s["opacities"] = np.full_like(s["opacities"], 0.995)
    cam = scenes.tiny_camera(250, 131)
    cam["cx"], cam["cy"] = 125.0, 65.5
    out = R.render(upload(s), cam)
    ref = oracle.render(s, cam)
    check_image(out, ref)
    assert (ref["T"] < 1e-4).mean() > 0.05


@pytest.mark.parametrize("size", [(16, 16), (13, 9), (1, 1), (17, 16)])
@pytest.mark.parametrize("mode", ["duplex", "alpha"])
def test_single_tile_and_tiny_images(R, size, mode):
    """One tile (no tile bits: the key sort has no pass and the lists stay
    where the emission put them, in depth order), a single pixel, and two
    tiles: lists bit-exact and pixels against the oracle."""
    w, h = size
    s = scenes.make_tiny_scene(1, n_cells=400, K=4)
    base = scenes.tiny_camera()
    cam = scenes.pinhole(base["viewmat"], w, h, fov_x_deg=12.0)
    out = R.render(upload(s), cam, mode=mode)
    ref = oracle.render(s, cam, mode=mode)
    check_image(out, ref)
    tiles = ((w + 15) // 16) * ((h + 15) // 16)
    keys, vals, ranges = R.read_lists(tiles)
    d = oracle.cells_discrete(s, cam) if mode == "duplex" else oracle.gauss_discrete(s, cam)
    ids, _, oranges = oracle.build_lists(d["visible"], d["depth_bits"], d["rect"], w, h)
    assert len(ids) > 0
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)


def test_k1_duplex_equals_alpha_blending_on_gpu(R):
    """K = 1, proxy = its Gaussian, kappa = 3, v = 1: C D (Duplex) equals the
    alpha-blended colour on black and D = 1 - T."""
    s = scenes.make_tiny_scene(0, n_cells=3000, K=1)
    s = dict(s, cell_pos=s["means"].copy(), cell_scale=s["scales"].copy(), cell_rot=s["rots"].copy())
    cam = scenes.tiny_camera()
    ds = upload(s)
    d = R.render(ds, cam, v_one=True, kappa=3.0)
    dc = (d["color"] * d["D"][None]).clone()
    dD = d["D"].clone()
    a = R.render(ds, cam, mode="alpha")
    diff = (dc - a["color"]).abs().max().item()
    assert diff <= 1e-5
    assert (dD - (1 - a["T"])).abs().max().item() <= 1e-5


@pytest.mark.parametrize("frame", [0, 30])
def test_1080p_sampled_pixels(R, c1, frame):
    """Full-size 1M-Gaussian scene at 1920x1080, in the benchmark's launch
    configuration; the oracle checks sampled pixels plus two whole tiles."""
    cam = scenes.orbit_cameras(60, 1920, 1080)[frame]
    out = R.render(upload(c1), cam)
    rng = np.random.default_rng(frame)
    pix = np.stack([rng.integers(0, 1920, 6000), rng.integers(0, 1080, 6000)], 1)
    tile = np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="xy"), -1).reshape(-1, 2)
    pix = np.concatenate([pix, tile + [960, 528], tile + [1904, 1072 - 8]], 0)
    pix = pix[(pix[:, 0] < 1920) & (pix[:, 1] < 1080)]
    ref = oracle.render(c1, cam, pixels=pix)
    col = out["color"].permute(1, 2, 0).double().cpu().numpy()[pix[:, 1], pix[:, 0]]
    err = oracle.admissible_max_err(col, ref)
    ok = np.isfinite(err)
    assert ok.mean() > 0.998
    assert np.nanmax(err) <= TOL, f"max abs error {np.nanmax(err):.3e}"
    assert (ref["D"] > 0).mean() > 0.5


@pytest.mark.parametrize("frame", [0, 30])
@pytest.mark.parametrize("mode", ["duplex", "alpha"])
def test_1080p_full_frame(R, c1, frame, mode):
    """Every pixel of orbit frames 0 and 30 of the 1M-Gaussian scene at
    1920x1080, in the benchmark's launch configuration, against the oracle:
    colour under the admissible-set rule, D and T within the tolerance and
    `last` equal on pixels without marginal decisions."""
    cam = scenes.orbit_cameras(60, 1920, 1080)[frame]
    out = R.render(upload(c1), cam, mode=mode)
    ref = oracle.render(c1, cam, mode=mode)
    check_image(out, ref)
    check_aux(out, ref)
    assert (ref["D"] > 0).mean() > 0.5


def test_1080p_alpha_mode_sampled_pixels(R, c1):
    cam = scenes.orbit_cameras(60, 1920, 1080)[10]
    out = R.render(upload(c1), cam, mode="alpha")
    rng = np.random.default_rng(7)
    pix = np.stack([rng.integers(0, 1920, 3000), rng.integers(0, 1080, 3000)], 1)
    ref = oracle.render(c1, cam, mode="alpha", pixels=pix)
    col = out["color"].permute(1, 2, 0).double().cpu().numpy()[pix[:, 1], pix[:, 0]]
    err = oracle.admissible_max_err(col, ref)
    assert np.isfinite(err).mean() > 0.998
    assert np.nanmax(err) <= TOL


def test_1080p_lcwsr_sampled_pixels(R, c1):
    cam = scenes.orbit_cameras(60, 1920, 1080)[20]
    out = R.render(upload(c1), cam, mode="lcwsr", tau=8.0)
    rng = np.random.default_rng(11)
    pix = np.stack([rng.integers(0, 1920, 3000), rng.integers(0, 1080, 3000)], 1)
    ref = oracle.render(c1, cam, mode="lcwsr", pixels=pix, tau=8.0)
    col = out["color"].permute(1, 2, 0).double().cpu().numpy()[pix[:, 1], pix[:, 0]]
    err = oracle.admissible_max_err(col, ref)
    assert np.isfinite(err).mean() > 0.998
    assert np.nanmax(err) <= TOL, f"max abs error {np.nanmax(err):.3e}"
    assert (ref["nrend"] == ref["nval"]).all()


# ------------------------------------------------------------------ edge cases

def test_empty_scene_and_all_culled(R):
    s = scenes.make_tiny_scene(0, n_cells=0, K=4)
    cam = scenes.tiny_camera(64, 48)
    out = R.render(upload(s), cam, bg=(0.1, 0.2, 0.3))
    assert torch.allclose(out["color"][1], torch.full_like(out["color"][1], 0.2))
    assert (out["D"] == 0).all() and (out["T"] == 1).all() and (out["last"] == 0).all()
    s2 = scenes.make_tiny_scene(0)
    cam2 = dict(cam)
    V = np.asarray(cam["viewmat"]).copy()
    V[:3, :3] = -V[:3, :3]  # camera looking away (det stays -1 * -1 ... only a cull test)
    V[2, 3] = -10.0
    cam2["viewmat"] = V
    out2 = R.render(upload(s2), cam2)
    assert (out2["D"] == 0).all()
    assert R.stats()["num_keys"] == 0


def test_capacity_overflow_is_reported_and_recovered(R):
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import Renderer
    r = Renderer(0)
    r.reserve(1000)
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    ds = upload(s)
    out = r.alloc_image(cam)
    from paper_2508_03180_amd.renderer import opts_struct
    _capi.check(r.render_into(ds, cam, out, opts_struct()), r.ctx)
    assert _capi.dgs_sync(r.ctx) == _capi.DGS_ERR_CAPACITY
    assert r.stats()["num_keys"] > 1000
    out = r.render(ds, cam)  # reserves and renders again
    ref = oracle.render(s, cam)
    check_image(out, ref)
    r.close()


def test_invalid_arguments_are_rejected(R):
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import camera_struct, opts_struct
    s = upload(scenes.make_tiny_scene(0))
    cam = scenes.tiny_camera()
    out = R.alloc_image(cam)
    bad = dict(cam, width=0)
    assert R.render_into(s, bad, out, opts_struct()) == _capi.DGS_ERR_INVALID_ARG
    bad = dict(cam, z_near=-1.0)
    assert R.render_into(s, bad, out, opts_struct()) == _capi.DGS_ERR_INVALID_ARG
    st = s.struct()
    st.gaussians_per_cell = 33
    img = _capi.dgs_image()
    img.color = out["color"].data_ptr()
    assert _capi.dgs_render(R.ctx, st, camera_struct(cam), opts_struct(), img) == _capi.DGS_ERR_INVALID_ARG
    assert "gaussians_per_cell" in _capi.dgs_last_error(R.ctx)
    assert R.render_into(s, cam, out, opts_struct(alpha_max=1.0)) == _capi.DGS_ERR_INVALID_ARG


def test_render_is_deterministic(R, c1):
    cam = scenes.orbit_cameras(60, 1920, 1080)[5]
    ds = upload(c1)
    a = R.render(ds, cam)["color"].clone()
    b = R.render(ds, cam)["color"].clone()
    assert torch.equal(a, b)


@pytest.mark.parametrize("mode", ["duplex", "lcwsr", "alpha"])
def test_one_stream_and_two_stream_frames_are_identical(R, c1, mode):
    """With stage timing on a frame runs on one stream; off, the member
    projection runs on a second stream beside the cell sort.  Both must give
    the same bits in every output, frame after frame."""
    from paper_2508_03180_amd import _capi
    cams = scenes.orbit_cameras(60, 1920, 1080)
    ds = upload(c1)
    opts = dict(mode=mode, tau=8.0) if mode == "lcwsr" else dict(mode=mode)
    for i in (3, 29):
        _capi.dgs_set_timing(R.ctx, 1)
        a = {k: v.clone() for k, v in R.render(ds, cams[i], **opts).items()}
        _capi.dgs_set_timing(R.ctx, 0)
        b = R.render(ds, cams[i], **opts)
        for k in ("color", "D", "T", "last"):
            assert torch.equal(a[k], b[k]), (mode, i, k)
    _capi.dgs_get_timing(R.ctx)


def test_stats_counters_match_oracle(R):
    """N^val and N^rendered (Sec. VII termination ratio) equal the oracle's
    sums; (pixel, cell) pairs reached equal the listed pairs without
    termination and lie between the contributing entries and that with it."""
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    ds = upload(s)
    R.render(ds, cam, stats=True)
    st = R.stats()
    ref = oracle.render(s, cam)
    exact = (ref["status"] == 0).all()
    if exact:
        assert st["n_val"] == int(ref["nval"].sum())
        assert st["n_rendered"] == int(ref["nrend"].sum())
    else:
        assert abs(st["n_val"] - int(ref["nval"].sum())) <= 8 * (ref["status"] != 0).sum()
    cd = oracle.cells_discrete(s, cam)
    _, _, ranges = oracle.build_lists(cd["visible"], cd["depth_bits"], cd["rect"], 256, 256)
    listed = int(((ranges[:, 1] - ranges[:, 0]) * 256).sum())  # 16x16 tiles, all inside the image
    R.render(ds, cam, stats=True, no_et=True)
    assert R.stats()["n_cell_pixels"] == listed
    assert int(ref["last"].sum()) <= st["n_cell_pixels"] < listed


# ------------------------------------------------------------------ ragged cells

@pytest.mark.parametrize("mode,kw", [("duplex", {}), ("lcwsr", dict(tau=4.5)), ("duplex", dict(no_et=True)),
                                     ("alpha", {})])
def test_ragged_cells_against_oracle(R, mode, kw):
    """Cells with their own member counts (0..32, CSR offsets): lists
    bit-exact, pixels within the tolerance, D, T and `last` on exact pixels;
    the cell modes also give the same bits as the scene padded to 32
    members per cell with invalid Gaussians."""
    s = scenes.make_ragged_scene(0)
    cam = scenes.tiny_camera()
    out = {k: v.clone() for k, v in R.render(upload(s), cam, mode=mode, **kw).items()}
    keys, vals, ranges = R.read_lists(256)
    d = oracle.cells_discrete(s, cam) if mode != "alpha" else oracle.gauss_discrete(s, cam)
    ids, _, oranges = oracle.build_lists(d["visible"], d["depth_bits"], d["rect"], 256, 256)
    assert keys.numel() == len(ids) > 1000
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)
    ref = oracle.render(s, cam, mode=mode, **kw)
    check_image(out, ref)
    check_aux(out, ref, d_rtol=1e-5 if mode == "lcwsr" else 0.0)
    if mode != "alpha":
        pad = R.render(upload(scenes.pad_to_fixed_k(s)), cam, mode=mode, **kw)
        for k in ("color", "D", "T", "last"):
            assert torch.equal(out[k], pad[k]), k


def test_ragged_cells_wide_view(R):
    """A 1280x720 view of a larger ragged scene (k_max 12): lists and pixels."""
    s = scenes.make_ragged_scene(5, n_cells=20_000, k_max=12, sh_degree=3)
    cam = scenes.pinhole(scenes.tiny_camera()["viewmat"], 1280, 720, fov_x_deg=50.0)
    out = R.render(upload(s), cam)
    cd = oracle.cells_discrete(s, cam)
    keys, vals, ranges = R.read_lists(80 * 45)
    ids, _, oranges = oracle.build_lists(cd["visible"], cd["depth_bits"], cd["rect"], 1280, 720)
    np.testing.assert_array_equal(vals.cpu().numpy(), ids)
    np.testing.assert_array_equal(ranges.cpu().numpy(), oranges)
    ref = oracle.render(s, cam)
    check_image(out, ref)
    check_aux(out, ref)


def test_malformed_offsets_are_reported(R):
    """A cell whose offsets run backwards, or claim more than K members, is
    culled on the device and dgs_sync reports DGS_ERR_INVALID_ARG; the other
    cells render as without it."""
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import opts_struct
    s = scenes.make_ragged_scene(2, n_cells=300, k_max=8)
    cam = scenes.tiny_camera()
    ds = upload(s)
    good = R.render(ds, cam)["color"].clone()
    offs = s["cell_offsets"].copy()
    n = int(np.nonzero(np.diff(offs) >= 2)[0][0])
    for bad in ("backwards", "too_many"):
        o = offs.copy()
        if bad == "backwards":
            o[n + 1] = o[n] - 1
        else:
            o[n + 1:] += 9  # cell n claims 9 + count members (> K = 8)
            o[-1] = offs[-1]
        ds.t["cell_offsets"] = torch.tensor(o, device="cuda")
        out = R.alloc_image(cam)
        _capi.check(R.render_into(ds, cam, out, opts_struct()), R.ctx)
        assert _capi.dgs_sync(R.ctx) == _capi.DGS_ERR_INVALID_ARG, bad
        assert "cell_offsets" in _capi.dgs_last_error(R.ctx)
        assert torch.isfinite(out["color"]).all()
    ds.t["cell_offsets"] = torch.tensor(offs, device="cuda")
    assert torch.equal(R.render(ds, cam)["color"], good)
