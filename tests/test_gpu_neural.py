"""Neural decode on the GPU against the oracle.

The decoded centres, scales and quaternions decide every Gaussian's pixel
box, so both sides compute them in binary32 in the same order and they must
match bit for bit; opacity and colour (continuous) within 1e-6.  The
rendered image of a neural scene must then match the oracle's render of the
oracle's own decode to the renderer's tolerance.
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


def upload(s, d):
    from paper_2508_03180_amd.renderer import NeuralDeviceScene
    return NeuralDeviceScene.from_numpy(s, d, "cuda:0")


def check_decoded(R, s, d, cam, visible):
    ref = oracle.decode(s, d, cam)
    got = {k: v.cpu().numpy() for k, v in R.read_decoded(s["cell_pos"].shape[0] * s["K"]).items()}
    g = np.repeat(visible.astype(bool), s["K"])
    assert g.sum() > 0
    for k in ("means", "scales", "rots"):
        np.testing.assert_array_equal(got[k][g], ref[k][g], err_msg=k)
    np.testing.assert_allclose(got["opacities"][g], ref["opacity64"][g], atol=1e-6)
    np.testing.assert_allclose(got["colors"][g], ref["color64"][g], atol=1e-6)
    return ref


def check_image(out, ref):
    col = out["color"].permute(1, 2, 0).reshape(-1, 3).double().cpu().numpy()
    err = oracle.admissible_max_err(col, ref)
    ok = np.isfinite(err)
    assert ok.mean() >= 0.999
    assert np.nanmax(err) <= TOL, f"max abs error {np.nanmax(err):.3e}"


@pytest.mark.parametrize("F,H,K", [(32, 32, 8), (16, 24, 5), (48, 64, 4)])
def test_decoded_attributes_and_image(R, F, H, K):
    s, d = scenes.make_neural_scene(5, n_cells=2500, K=K, F=F, H=H)
    cam = scenes.orbit_cameras(12, 320, 240)[2]
    ns = upload(s, d)
    out = R.render_neural(ns, cam)
    cd = oracle.cells_discrete(s, cam)
    ref_scene = check_decoded(R, s, d, cam, cd["visible"])
    ref = oracle.render(ref_scene, cam)
    check_image(out, ref)
    # pixel boxes of the decoded Gaussians
    gr = R.read_gauss_rects(ns.M).cpu().numpy()
    gd = oracle.gauss_discrete(ref_scene, cam)
    proj = np.repeat(cd["visible"].astype(bool), K)
    np.testing.assert_array_equal(gr[proj], gd["rect"][proj])


@pytest.mark.parametrize("opts", [dict(mode="alpha"), dict(mode="lcwsr", tau=5.0), dict(v_one=True, bg=(0.2, 0.3, 0.4))])
def test_neural_modes(R, opts):
    s, d = scenes.make_neural_scene(6, n_cells=2000, K=6)
    cam = scenes.orbit_cameras(12, 256, 256)[7]
    out = R.render_neural(upload(s, d), cam, **opts)
    vis = np.ones(len(s["cell_pos"]), bool) if opts.get("mode") == "alpha" else \
        oracle.cells_discrete(s, cam)["visible"]
    ref_scene = check_decoded(R, s, d, cam, vis)
    check_image(out, oracle.render(ref_scene, cam, **opts))


def test_neural_1080p_sampled_pixels(R):
    """The benchmark-size neural scene (100,000 cells x 10) at 1920x1080."""
    s, d = scenes.make_neural_scene(1)
    cam = scenes.orbit_cameras(60, 1920, 1080)[5]
    out = R.render_neural(upload(s, d), cam)
    cd = oracle.cells_discrete(s, cam)
    ref_scene = check_decoded(R, s, d, cam, cd["visible"])
    rng = np.random.default_rng(2)
    pix = np.stack([rng.integers(0, 1920, 4000), rng.integers(0, 1080, 4000)], 1)
    ref = oracle.render(ref_scene, cam, pixels=pix)
    col = out["color"].permute(1, 2, 0).double().cpu().numpy()[pix[:, 1], pix[:, 0]]
    err = oracle.admissible_max_err(col, ref)
    assert np.isfinite(err).mean() > 0.998
    assert np.nanmax(err) <= TOL


def test_neural_arguments_and_no_backward(R):
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import camera_struct, opts_struct
    s, d = scenes.make_neural_scene(7, n_cells=100, K=4, F=8, H=8)
    ns = upload(s, d)
    cam = scenes.orbit_cameras(12, 64, 64)[0]
    out = R.alloc_image(cam)
    img = _capi.dgs_image(out["color"].data_ptr(), None, None, None)
    bad = ns.decoder_struct()
    bad.feature_dim = 65
    assert _capi.dgs_render_neural(R.ctx, ns.struct(), bad, camera_struct(cam), opts_struct(), img) == \
        _capi.DGS_ERR_INVALID_ARG
    bad = ns.decoder_struct()
    bad.weights = None
    assert _capi.dgs_render_neural(R.ctx, ns.struct(), bad, camera_struct(cam), opts_struct(), img) == \
        _capi.DGS_ERR_INVALID_ARG
    R.render_neural(ns, cam, out=out)
    # a neural render saves no frame (dgs_render_neural has no `saved`
    # argument), so there is nothing a backward could replay
    import inspect
    assert "saved" not in inspect.signature(_capi.dgs_render_neural).parameters
