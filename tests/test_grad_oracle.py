"""Pins of the binary64 gradient oracle (oracle/grad.py), CPU only."""
import numpy as np
import pytest
import torch

import oracle
from oracle import grad as go
from paper_2508_03180_amd import scenes


def small_case():
    s = scenes.make_tiny_scene(0, n_cells=400, K=6)
    s["sh"] = np.concatenate([s["sh"], np.random.default_rng(1).normal(0, 0.3, (s["sh"].shape[0], 15, 3))],
                             1).astype(np.float32)
    s["sh_degree"] = 3
    cam = scenes.tiny_camera(64, 64)
    pix = np.stack(np.meshgrid(np.arange(64), np.arange(64), indexing="xy"), -1).reshape(-1, 2)
    return s, cam, pix


def test_forward_equals_c_oracle():
    s, cam, pix = small_case()
    fz = go.FrozenScene(s, cam)
    p = go.params_from_scene(s, requires_grad=False)
    C, D, T = go.render(p, fz, pix)
    ref = oracle.render(s, cam, pixels=pix)
    ok = ref["status"] == 0
    assert ok.mean() > 0.99 and (ref["D"] > 0).mean() > 0.3
    np.testing.assert_allclose(C.numpy()[ok], ref["color"][ok], atol=1e-11)
    np.testing.assert_allclose(D.numpy()[ok], ref["D"][ok], atol=1e-11)
    np.testing.assert_allclose(T.numpy()[ok], ref["T"][ok], atol=1e-11)


@pytest.mark.parametrize("flags", [dict(), dict(v_one=True)])
def test_autograd_equals_finite_differences_of_frozen_forward(flags):
    """Directional derivatives along random directions, h = 1e-6 (decisions
    stay frozen within such steps)."""
    s, cam, pix = small_case()
    fz = go.FrozenScene(s, cam)
    rng = np.random.default_rng(2)
    gC = torch.tensor(rng.standard_normal((pix.shape[0], 3)))
    gD = torch.tensor(rng.standard_normal(pix.shape[0]))

    def loss(p, masks=False):
        C, D, _, m = go.render(p, fz, pix, return_masks=True, **flags)
        L = (C * gC).sum() + (D * gD).sum()
        return (L, m) if masks else L

    p = go.params_from_scene(s)
    loss(p).backward()
    checked = 0
    for key in ("means", "scales", "rots", "opacities", "sh", "cell_v_sh", "cell_pos"):
        if flags.get("v_one") and key in ("cell_v_sh", "cell_pos"):
            continue
        for trial in range(4):
            # sparse direction: a few entries, so gate flips are rare and detected
            d = torch.zeros(p[key].shape, dtype=torch.float64)
            flat = d.view(-1)
            idx = rng.choice(flat.numel(), size=min(8, flat.numel()), replace=False)
            flat[torch.from_numpy(idx)] = torch.tensor(rng.standard_normal(len(idx)))
            h = 1e-7
            with torch.no_grad():
                pp = {k: v.detach().clone() for k, v in p.items()}
                pm = {k: v.detach().clone() for k, v in p.items()}
                pp[key] += h * d
                pm[key] -= h * d
                Lp, mp = loss(pp, True)
                Lm, mm = loss(pm, True)
            if not all(torch.equal(x, y) for x, y in zip(mp, mm)):
                continue  # a frozen decision moved inside the stencil
            fd = (Lp - Lm).item() / (2 * h)
            an = (p[key].grad * d).sum().item()
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (key, fd, an)
            checked += 1
    assert checked >= 12


def test_c_oracle_finite_differences_eps_1e3():
    """Central differences (eps = 1e-3) of the binary64 C oracle on single
    parameters agree with the autograd gradient wherever no discrete decision
    (box, tile list, alpha_min gate, termination) moves between the two
    stencil points.  Scales (about 0.01) take the step in log space."""
    s, cam, pix = small_case()
    rng = np.random.default_rng(3)
    gC = rng.standard_normal((pix.shape[0], 3))
    g = go.gradients(s, cam, pix, gC)

    def run(sc):
        r = oracle.render(sc, cam, pixels=pix, band_alpha=0.0, band_T=0.0)
        return float((r["color"] * gC).sum()), r["nrend"], r["last"], oracle.gauss_discrete(sc, cam)["rect"]

    gd0 = oracle.gauss_discrete(s, cam)
    vis = np.nonzero(gd0["visible"])[0]
    checked = 0
    for trial in range(80):
        key = ["means", "opacities", "sh", "scales", "cell_v_sh", "rots"][trial % 6]
        arr = s[key]
        if key == "cell_v_sh":
            idx = (int(rng.integers(0, arr.shape[0])), int(rng.integers(0, arr.shape[1])))
        else:
            gi = int(rng.choice(vis))
            idx = (gi,) + tuple(int(rng.integers(0, n)) for n in arr.shape[1:])
        eps = 1e-3
        sp, sm = dict(s), dict(s)
        sp[key] = arr.copy(); sm[key] = arr.copy()
        if key == "scales":
            sp[key][idx] *= np.exp(eps); sm[key][idx] *= np.exp(-eps)
            step = float(np.log(sp[key][idx]) - np.log(sm[key][idx]))
            an = float(g[key][idx]) * float(arr[idx])  # dL/dlog s
        else:
            sp[key][idx] += eps; sm[key][idx] -= eps
            step = float(sp[key][idx]) - float(sm[key][idx])  # float32-rounded stencil width
            an = float(g[key][idx])
        Lp, np_, lp, rp = run(sp)
        Lm, nm, lm, rm = run(sm)
        if not (np.array_equal(np_, nm) and np.array_equal(lp, lm) and np.array_equal(rp, gd0["rect"])
                and np.array_equal(rm, gd0["rect"])):
            continue  # a discrete decision moved inside the stencil
        fd = (Lp - Lm) / step
        if abs(an) < 1e-3 and abs(fd) < 1e-3:
            continue
        assert abs(fd - an) <= 1e-2 * max(abs(an), 1e-2), (key, idx, fd, an)
        checked += 1
    assert checked >= 15


def test_ragged_cells_gradient_equals_padded_scene():
    """Variable member counts (CSR offsets): the forward equals the C oracle
    and the gradient of every Gaussian equals that of its copy in the same
    scene padded to 32 members per cell with invalid Gaussians (which get
    exactly zero)."""
    s = scenes.make_ragged_scene(3, n_cells=300, sh_degree=1)
    cam = scenes.tiny_camera(64, 64)
    pix = np.stack(np.meshgrid(np.arange(64), np.arange(64), indexing="xy"), -1).reshape(-1, 2)
    fz = go.FrozenScene(s, cam)
    C, D, T = go.render(go.params_from_scene(s, requires_grad=False), fz, pix)
    ref = oracle.render(s, cam, pixels=pix)
    ok = ref["status"] == 0
    assert (ref["D"] > 0).mean() > 0.3
    np.testing.assert_allclose(C.numpy()[ok], ref["color"][ok], atol=1e-11)
    rng = np.random.default_rng(0)
    gC = rng.standard_normal((pix.shape[0], 3))
    gD = rng.standard_normal(pix.shape[0])
    a = go.gradients(s, cam, pix, gC, gD)
    p = scenes.pad_to_fixed_k(s)
    b = go.gradients(p, cam, pix, gC, gD)
    offs = s["cell_offsets"].astype(np.int64)
    counts = np.diff(offs)
    have = (np.arange(32)[None, :] < counts[:, None]).reshape(-1)
    for k in ("means", "scales", "rots", "opacities", "sh"):
        np.testing.assert_allclose(b[k][have], a[k], rtol=1e-12, atol=1e-14, err_msg=k)
        assert np.all(b[k][~have] == 0), k
    for k in ("cell_v_sh", "cell_pos"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-12, atol=1e-14, err_msg=k)
    assert np.abs(a["means"]).max() > 0
