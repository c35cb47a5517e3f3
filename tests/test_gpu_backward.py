"""GPU backward of the hybrid renderer against the binary64 gradient oracle.

The loss is the linear functional L = sum gC . C + sum gD . D with random
weights (its gradient is the vector-Jacobian product of the renderer).  Per
parameter group the GPU gradient must match the oracle's to a relative L2
error below 1e-3 and a cosine similarity above 0.9999 (float32 against
binary64; rare alpha_min / termination decisions that fall within rounding
of their threshold can differ and contribute the residual).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import grad as go
from paper_2508_03180_amd import scenes

pytestmark = pytest.mark.gpu

GROUPS = ("means", "scales", "rots", "opacities", "sh", "cell_v_sh", "cell_pos")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2508_03180_amd.renderer import Renderer
    r = Renderer(0)
    yield r
    r.close()


def natural(g, key, shape):
    t = g[key]
    if key == "sh":
        return t.permute(2, 0, 1).reshape(shape).double().cpu().numpy()
    if key == "opacities":
        return t.double().cpu().numpy()
    return t.t().reshape(shape).double().cpu().numpy()


def compare(gpu, ref, scene):
    out = {}
    for k in GROUPS:
        a = natural(gpu, k, scene[k].shape).ravel()
        b = ref[k].ravel()
        nb = np.linalg.norm(b)
        if nb == 0:
            assert np.linalg.norm(a) < 1e-6
            continue
        rel = np.linalg.norm(a - b) / nb
        cos = float(a @ b / (np.linalg.norm(a) * nb + 1e-300))
        out[k] = (rel, cos)
    return out


def run_case(R, s, cam, pixels_mask, seed=0, **opts):
    from paper_2508_03180_amd.renderer import DeviceScene
    H, W = cam["height"], cam["width"]
    rng = np.random.default_rng(seed)
    gC = rng.standard_normal((3, H, W)) * pixels_mask[None]
    gD = rng.standard_normal((H, W)) * pixels_mask
    ds = DeviceScene.from_numpy(s, "cuda:0")
    out = R.render(ds, cam, save=True, **opts)
    g = R.render_backward(ds, out["frame"], torch.tensor(gC, dtype=torch.float32, device="cuda"),
                          torch.tensor(gD, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    out["frame"].release()
    ys, xs = np.nonzero(pixels_mask)
    pix = np.stack([xs, ys], 1)
    ref = go.gradients(s, cam, pix, gC[:, ys, xs].T, gD[ys, xs], **opts)
    return compare(g, ref, s)


def small_scene():
    s = scenes.make_tiny_scene(0, n_cells=400, K=6)
    s["sh"] = np.concatenate([s["sh"], np.random.default_rng(1).normal(0, 0.3, (s["sh"].shape[0], 15, 3))],
                             1).astype(np.float32)
    s["sh_degree"] = 3
    return s


def check(res):
    for k, (rel, cos) in res.items():
        assert rel < 1e-3 and cos > 0.9999, (k, rel, cos)


def test_backward_small_scene_whole_image(R):
    s = small_scene()
    cam = scenes.tiny_camera(64, 64)
    check(run_case(R, s, cam, np.ones((64, 64))))


@pytest.mark.parametrize("opts", [dict(v_one=True), dict(no_et=True), dict(bg=(0.3, 0.2, 0.1))])
def test_backward_options(R, opts):
    s = small_scene()
    cam = scenes.tiny_camera(64, 64)
    check(run_case(R, s, cam, np.ones((64, 64)), seed=4, **opts))


def test_backward_tiny_scene_window(R):
    s = scenes.make_tiny_scene(0)
    cam = scenes.tiny_camera()
    m = np.zeros((256, 256))
    m[96:160, 96:160] = 1
    check(run_case(R, s, cam, m, seed=1))


def test_backward_opaque_scene_with_termination(R):
    s = small_scene()
    s["opacities"] = np.full_like(s["opacities"], 0.97)
    cam = scenes.tiny_camera(64, 64)
    check(run_case(R, s, cam, np.ones((64, 64)), seed=2))


def test_zero_weight_cells_forward_and_backward(R):
    """Cells whose weight v underflows to 0 in binary32 (logit -282) add
    nothing and leave the gates of every other cell unchanged; the forward
    and the backward stay finite.  Pixels whose weight sum D the oracle puts
    below 1e-3 are left out of the comparison: where only such cells
    contribute, C = N / D divides binary64 weights of ~1e-123 (the oracle's
    colour) while binary32 has D = 0 (the background)."""
    import oracle
    from paper_2508_03180_amd.renderer import DeviceScene
    s = small_scene()
    v = s["cell_v_sh"].copy()
    v[::3, 0] = -1000.0
    s["cell_v_sh"] = v
    cam = scenes.tiny_camera(64, 64)
    out = R.render(DeviceScene.from_numpy(s, "cuda:0"), cam)
    col = out["color"].permute(1, 2, 0).reshape(-1, 3).double().cpu().numpy()
    assert np.isfinite(col).all()
    ref = oracle.render(s, cam)
    keep = ref["D"] >= 1e-3
    assert keep.mean() > 0.3
    err = oracle.admissible_max_err(col, ref)[keep]
    assert np.isfinite(err).mean() >= 0.999
    assert np.nanmax(err) <= 2e-4
    check(run_case(R, s, cam, keep.reshape(64, 64).astype(np.float64), seed=5))


@pytest.mark.parametrize("seed", [1, 2])
def test_backward_tiles_at_the_split_length(R, seed):
    """Gradients of the pixels of tiles whose cell lists are one short of,
    exactly at and one past the length at which the compositor splits a
    tile into two half-tile items (32 cells); the backward replays the
    forward's items."""
    import oracle
    s = scenes.make_tiny_scene(seed)
    cam = scenes.tiny_camera()
    d = oracle.cells_discrete(s, cam)
    _, _, ranges = oracle.build_lists(d["visible"], d["depth_bits"], d["rect"], 256, 256)
    lens = ranges[:, 1] - ranges[:, 0]
    tiles = np.nonzero((lens >= 31) & (lens <= 33))[0]
    assert len(tiles) > 0
    m = np.zeros((256, 256))
    for t in tiles:
        ty, tx = divmod(int(t), 16)
        m[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = 1
    check(run_case(R, s, cam, m, seed=6))


def test_backward_1080p_window(R):
    """Full-size 1M-Gaussian scene at 1920x1080 (the benchmark's launch
    configuration); the oracle takes the loss on a 48x48 window."""
    s = scenes.make_mid_scene(1)
    cam = scenes.orbit_cameras(60, 1920, 1080)[0]
    m = np.zeros((1080, 1920))
    m[500:548, 930:978] = 1
    check(run_case(R, s, cam, m, seed=3))


def test_autograd_function_matches_direct_backward(R):
    from paper_2508_03180_amd.renderer import DuplexRender
    s = small_scene()
    cam = scenes.tiny_camera(64, 64)
    t = {k: torch.tensor(s[k], device="cuda", requires_grad=True)
         for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "means", "scales", "rots", "opacities", "sh")}
    C, D = DuplexRender.apply(R, cam, {}, t["cell_pos"], t["cell_scale"], t["cell_rot"], t["cell_v_sh"],
                              t["means"], t["scales"], t["rots"], t["opacities"], t["sh"])
    wC = torch.randn_like(C)
    wD = torch.randn_like(D)
    ((C * wC).sum() + (D * wD).sum()).backward()
    ys, xs = np.mgrid[0:64, 0:64]
    pix = np.stack([xs.ravel(), ys.ravel()], 1)
    ref = go.gradients(s, cam, pix, wC.permute(1, 2, 0).reshape(-1, 3).double().cpu().numpy(),
                       wD.reshape(-1).double().cpu().numpy())
    for k in GROUPS:
        a = t[k].grad.double().cpu().numpy().ravel()
        b = ref[k].ravel()
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b), k
    assert t["cell_scale"].grad is None and t["cell_rot"].grad is None
    # other renders between the forward and the backward change nothing
    t2 = {k: torch.tensor(s[k], device="cuda", requires_grad=True) for k in t}
    C2, D2 = DuplexRender.apply(R, cam, {}, t2["cell_pos"], t2["cell_scale"], t2["cell_rot"], t2["cell_v_sh"],
                                t2["means"], t2["scales"], t2["rots"], t2["opacities"], t2["sh"])
    R.render(__import__("paper_2508_03180_amd.renderer", fromlist=["DeviceScene"]).DeviceScene.from_numpy(
        scenes.make_tiny_scene(5), "cuda:0"), scenes.tiny_camera(), save=True)
    ((C2 * wC).sum() + (D2 * wD).sum()).backward()
    for k in GROUPS:
        torch.testing.assert_close(t2[k].grad, t[k].grad, rtol=1e-5, atol=1e-6, msg=k)


def test_backward_rejects_alpha_mode_and_mismatch(R):
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import DeviceScene, camera_struct, opts_struct
    s = small_scene()
    cam = scenes.tiny_camera(64, 64)
    ds = DeviceScene.from_numpy(s, "cuda:0")
    for mode, kw in (("alpha", {}), ("lcwsr", dict(tau=4.0))):
        with pytest.raises(_capi.DgsError, match="UNSUPPORTED"):
            R.render(ds, cam, mode=mode, save=True, **kw)
    out = R.render(ds, cam, save=True)
    fr = out["frame"]
    gC = torch.zeros((3, 64, 64), device="cuda")
    g = R.render_backward(ds, fr, gC)
    gr = _capi.dgs_grads()
    for k, a in (("means", "d_means"), ("scales", "d_scales"), ("rots", "d_rots"), ("opacities", "d_opacities"),
                 ("sh", "d_sh"), ("cell_v_sh", "d_cell_v_sh"), ("cell_pos", "d_cell_pos")):
        setattr(gr, a, g[k].data_ptr())
    gr.overwrite = 1

    def bwd(scene, cam_, opts_):
        return _capi.dgs_render_backward(R.ctx, scene, cam_, opts_, fr.handle, gC.data_ptr(), None, gr)
    assert bwd(ds.struct(), None, None) == _capi.DGS_OK
    assert bwd(ds.struct(), camera_struct(cam), opts_struct()) == _capi.DGS_OK
    assert bwd(ds.struct(), camera_struct(cam), opts_struct(stats=True)) == _capi.DGS_OK
    assert bwd(ds.struct(), camera_struct(dict(cam, fx=cam["fx"] * 1.01)), None) == _capi.DGS_ERR_INVALID_ARG
    assert "camera" in _capi.dgs_last_error(R.ctx)
    assert bwd(ds.struct(), None, opts_struct(v_one=True)) == _capi.DGS_ERR_INVALID_ARG
    assert bwd(ds.struct(), None, opts_struct(mode="alpha")) == _capi.DGS_ERR_UNSUPPORTED
    other = DeviceScene.from_numpy(scenes.make_tiny_scene(0, n_cells=401, K=6), "cuda:0")
    assert bwd(other.struct(), None, None) == _capi.DGS_ERR_INVALID_ARG
    assert "sizes" in _capi.dgs_last_error(R.ctx)
    # alpha_max must stay below 1 (every factor 1 - v alpha > 0)
    assert R.render_into(ds, cam, R.alloc_image(cam), opts_struct(alpha_max=1.0)) == _capi.DGS_ERR_INVALID_ARG
    fr.release()
    assert bwd(ds.struct(), None, None) == _capi.DGS_ERR_INVALID_ARG  # released
    assert _capi.dgs_frame_release(R.ctx, fr.handle or _capi.dgs_frame(0)) == _capi.DGS_ERR_INVALID_ARG
    torch.cuda.synchronize()


@pytest.mark.parametrize("v_one", [False, True])
def test_overwrite_and_accumulate_modes_agree(R, v_one):
    """Written gradients (buffers full of NaN beforehand, never read) equal
    gradients added into zeroed buffers, and a second backward doubles
    them; every entry is written, including Gaussians and cells that get no
    gradient."""
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import DeviceScene, camera_struct, opts_struct
    s = small_scene()
    # a narrow view: cells outside it get no gradient
    cam = scenes.pinhole(scenes.tiny_camera()["viewmat"], 64, 64, fov_x_deg=25.0)
    ds = DeviceScene.from_numpy(s, "cuda:0")
    opts = dict(v_one=True) if v_one else {}
    out = R.render(ds, cam, save=True, **opts)
    fr = out["frame"]
    gC = torch.randn((3, 64, 64), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    g = R.render_backward(ds, fr, gC, mean2d=True)
    # overwrite into NaN-filled buffers through the C ABI
    nan = {k: torch.full_like(v, float("nan")) for k, v in g.items()}
    gr = _capi.dgs_grads()
    gr.d_means, gr.d_scales, gr.d_rots = nan["means"].data_ptr(), nan["scales"].data_ptr(), nan["rots"].data_ptr()
    gr.d_opacities, gr.d_sh = nan["opacities"].data_ptr(), nan["sh"].data_ptr()
    gr.d_cell_v_sh, gr.d_cell_pos, gr.d_mean2d = (nan["cell_v_sh"].data_ptr(), nan["cell_pos"].data_ptr(),
                                                  nan["mean2d"].data_ptr())
    gr.overwrite = 1
    _capi.check(_capi.dgs_render_backward(R.ctx, ds.struct(), camera_struct(cam), opts_struct(**opts), fr.handle,
                                          gC.data_ptr(), None, gr), R.ctx)
    acc = {k: torch.zeros_like(v) for k, v in g.items()}
    R.render_backward(ds, fr, gC, into=acc)
    torch.cuda.synchronize()
    for k in g:
        assert not torch.isnan(nan[k]).any(), k
        torch.testing.assert_close(nan[k], g[k], rtol=1e-5, atol=1e-7, msg=k)
        torch.testing.assert_close(acc[k], g[k], rtol=1e-5, atol=1e-7, msg=k)
    R.render_backward(ds, fr, gC, into=acc)
    torch.cuda.synchronize()
    for k in g:
        torch.testing.assert_close(acc[k], 2 * g[k], rtol=1e-5, atol=1e-7, msg=k)
    fr.release()
    # Gaussians and cells outside the view get no gradient: zeros
    assert (g["means"].abs().sum(0) == 0).any() and (g["sh"].abs().sum((0, 1)) == 0).any()
    if v_one:
        assert (g["cell_v_sh"] == 0).all() and (g["cell_pos"] == 0).all()


def test_low_weight_cells_forward_and_backward(R):
    """Cells with v logits between -12 and -20 (v from 6e-6 down to 2e-9):
    1 - v alpha rounds to 1 in binary32, yet such a cell still contributes
    v T A to N and v T B to D.  It must count as contributing (`last`
    equal to the oracle's on every pixel without marginal decisions) and its
    members and v must get their gradient, also where only such cells
    cover a pixel."""
    import oracle
    from paper_2508_03180_amd.renderer import DeviceScene
    s = small_scene()
    rng = np.random.default_rng(12)
    v = s["cell_v_sh"].copy()
    low = rng.random(v.shape[0]) < 0.5
    v[low, 0] = rng.uniform(-20.0, -12.0, low.sum()) / (0.5 / np.sqrt(np.pi))
    v[low, 1:] = 0.0
    s["cell_v_sh"] = v
    cam = scenes.tiny_camera(64, 64)
    ds = DeviceScene.from_numpy(s, "cuda:0")
    out = R.render(ds, cam)
    ref = oracle.render(s, cam)
    exact = ref["status"] == 0
    last = out["last"].reshape(-1).cpu().numpy()
    np.testing.assert_array_equal(last[exact], ref["last"][exact])
    col = out["color"].permute(1, 2, 0).reshape(-1, 3).double().cpu().numpy()
    err = oracle.admissible_max_err(col, ref)
    assert np.isfinite(err).mean() >= 0.999 and np.nanmax(err) <= 2e-4
    # pixels covered by low-weight cells alone (D below 1e-4) exist and reach the backward
    assert ((ref["D"] > 0) & (ref["D"] < 1e-4)).sum() > 20
    res = run_case(R, s, cam, np.ones((64, 64)), seed=8)
    check(res)


@pytest.mark.parametrize("alpha_max", [0.99, 0.999])
def test_many_opaque_members_per_cell(R, alpha_max):
    """K = 32 members per cell, all near-opaque and overlapping, v = 1:
    a cell's product prod (1 - alpha) reaches (1 - alpha_max)^32, far below
    the binary32 range.  The backward must stay finite and match the oracle
    gradient (it never divides by such a product)."""
    from paper_2508_03180_amd.renderer import DeviceScene
    s = scenes.make_tiny_scene(4, n_cells=120, K=32)
    s["opacities"] = np.full_like(s["opacities"], 1.0)
    # members collapsed towards their cell centre, so that they overlap
    rep = np.repeat(s["cell_pos"], 32, 0)
    s["means"] = (rep + 0.05 * (s["means"] - rep)).astype(np.float32)
    s["scales"] = (s["scales"] * 4.0).astype(np.float32)
    cam = scenes.tiny_camera(64, 64)
    for opts in (dict(v_one=True, alpha_max=alpha_max), dict(alpha_max=alpha_max, no_et=True, v_one=True)):
        ds = DeviceScene.from_numpy(s, "cuda:0")
        out = R.render(ds, cam, save=True, **opts)
        assert (out["T"] < 1e-30).float().mean().item() > 0.005  # products underflow on some pixels
        g = R.render_backward(ds, out["frame"], torch.ones((3, 64, 64), device="cuda"))
        torch.cuda.synchronize()
        for k, t in g.items():
            assert torch.isfinite(t).all(), (opts, k)
        check(run_case(R, s, cam, np.ones((64, 64)), seed=9, **opts))


def test_two_pending_frames_on_one_context(R):
    """Two saved renders, then their two backwards, on one context give the
    gradients each frame gets alone on a context of its own; a reserve and a
    sort between them do not disturb the saved frames."""
    from paper_2508_03180_amd.renderer import DeviceScene, Renderer
    s = small_scene()
    cams = [scenes.tiny_camera(64, 64), scenes.pinhole(scenes.tiny_camera()["viewmat"], 48, 40, fov_x_deg=40.0)]
    ds = DeviceScene.from_numpy(s, "cuda:0")
    gen = torch.Generator("cuda").manual_seed(3)
    gCs = [torch.randn((3, c["height"], c["width"]), device="cuda", generator=gen) for c in cams]
    solo = []
    for cam, gC in zip(cams, gCs):
        r = Renderer(0)
        out = r.render(ds, cam, save=True)
        solo.append({k: v.clone() for k, v in r.render_backward(ds, out["frame"], gC).items()})
        torch.cuda.synchronize()
        out["frame"].release()
        r.close()
    outs = [R.render(ds, cam, save=True) for cam in cams]
    R.reserve(4_000_000, 500_000, 20_000)  # grows (moves) the context's own buffers
    kt = torch.arange(1000, 0, -1, dtype=torch.int64, device="cuda")
    R.sort_pairs(kt, torch.arange(1000, dtype=torch.int32, device="cuda"), 16)
    for i in (1, 0):
        g = R.render_backward(ds, outs[i]["frame"], gCs[i])
        torch.cuda.synchronize()
        for k in g:
            torch.testing.assert_close(g[k], solo[i][k], rtol=1e-5, atol=1e-6, msg=(i, k))
    st = outs[0]["frame"].stats()
    assert st["num_keys"] > 0
    for o in outs:
        o["frame"].release()


def test_planar_autograd_function(R):
    """DuplexRenderPlanar: the same gradients as the natural-layout function,
    on planar leaves used in place."""
    from paper_2508_03180_amd.renderer import DuplexRender, DuplexRenderPlanar
    s = small_scene()
    cam = scenes.tiny_camera(64, 64)
    keys = ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "means", "scales", "rots", "opacities", "sh")
    nat = {k: torch.tensor(s[k], device="cuda", requires_grad=True) for k in keys}

    def planar(k, a):
        a = np.asarray(a, np.float32)
        if k == "sh":
            return np.ascontiguousarray(a.transpose(1, 2, 0))
        if k == "opacities":
            return a
        return np.ascontiguousarray(a.reshape(a.shape[0], -1).T)
    pl = {k: torch.tensor(planar(k, s[k]), device="cuda", requires_grad=True) for k in keys}
    C, D = DuplexRender.apply(R, cam, {}, *[nat[k] for k in keys])
    Cp, Dp = DuplexRenderPlanar.apply(R, cam, {}, *[pl[k] for k in keys])
    assert torch.equal(C, Cp) and torch.equal(D, Dp)
    wC, wD = torch.randn_like(C), torch.randn_like(D)
    ((C * wC).sum() + (D * wD).sum()).backward()
    ((Cp * wC).sum() + (Dp * wD).sum()).backward()
    for k in keys:
        if k in ("cell_scale", "cell_rot"):
            assert nat[k].grad is None and pl[k].grad is None
            continue
        want = torch.tensor(planar(k, nat[k].grad.cpu().numpy()), device="cuda")
        torch.testing.assert_close(pl[k].grad, want, rtol=1e-5, atol=1e-6, msg=k)


def test_backward_ragged_cells(R):
    """Cells with their own member counts (CSR offsets, 0..32 members):
    gradients against the binary64 oracle."""
    s = scenes.make_ragged_scene(3, n_cells=300, sh_degree=1)
    cam = scenes.tiny_camera(64, 64)
    check(run_case(R, s, cam, np.ones((64, 64)), seed=10))

