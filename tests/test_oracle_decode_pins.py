"""Pins of the oracle's neural decode (CPU only).

The decode follows the neural-Gaussian formulation (Sec. III-A) with the
cell proxy of Sec. IV-A: four MLPs F_sigma (tanh), F_c, F_s (sigmoid ratio)
and F_q of (f_n, delta_n, d_n); centres mu = x_n + R(Q_n)(O^pos * S_n) (eq.
scaffold_offset, offsets in the cell frame); scales s = r * S_n with
r = min(sigmoid(y_s), 1 - |O^pos|) (eqs. nerual_scales, scale_res).  These
tests check it against a hand-worked cell, binary64 re-evaluation in numpy,
closed forms of degenerate weights and the containment the clamps promise.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2508_03180_amd import scenes

A = oracle.DECODER_OUTPUTS


def unpack(w, F, H, K):
    """Split packed weights into per-decoder (W1, b1, W2, b2) in float64."""
    out, o = [], 0
    I = F + 4
    for a in A:
        O = K * a
        W1 = w[o:o + I * H].reshape(I, H); o += I * H
        b1 = w[o:o + H]; o += H
        W2 = w[o:o + H * O].reshape(H, O); o += H * O
        b2 = w[o:o + O]; o += O
        out.append(tuple(x.astype(np.float64) for x in (W1, b1, W2, b2)))
    assert o == w.size
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, np.float64).ravel() for d in parts for p in d]).astype(np.float32)


def axis_cam():
    return dict(viewmat=np.eye(4, dtype=np.float32), fx=100.0, fy=100.0, cx=50.0, cy=50.0, width=100, height=100,
                z_near=0.2)


def one_cell(pos=(0.0, 0.0, 2.0), scale=(0.1, 0.2, 0.3), offset=(0.6, 0.0, 0.0), feat=(1.0,)):
    return dict(cell_pos=np.array([pos], np.float32), cell_scale=np.array([scale], np.float32),
                cell_rot=np.array([[1, 0, 0, 0]], np.float32), cell_v_sh=np.zeros((1, 4), np.float32),
                v_sh_degree=1, K=1, features=np.array([feat], np.float32), offsets=np.array([offset], np.float32))


def test_exp32_accuracy():
    """The decode's binary32 exp is within 3 ulp of exp over its range and
    exact where the reduction leaves r = 0."""
    x = np.linspace(-87.0, 87.0, 200_001).astype(np.float32)
    got = oracle.exp32(x).astype(np.float64)
    ref = np.exp(x.astype(np.float64))
    ulp = np.spacing(ref.astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got - ref) / ulp) <= 3.0
    assert oracle.exp32(np.array([0.0], np.float32))[0] == 1.0
    for n in (-10, 1, 7):
        assert oracle.exp32(np.array([n * math.log(2)], np.float32))[0] == pytest.approx(2.0 ** n, rel=3e-7)


def test_hand_worked_cell():
    """F = H = K = 1, camera at the origin looking down +z, cell at (0,0,2):
    delta = 2 and d = (0,0,1), so each decoder's hidden unit and outputs can
    be worked by hand; the input order is (f, delta, d_x, d_y, d_z)."""
    # opacity: h = relu(f + 0.5 delta + 0.25 d_z) = 2.25; y = -4 + 2 h = 0.5
    dec_o = ([[1.0], [0.5], [0.0], [0.0], [0.25]], [0.0], [[2.0]], [-4.0])
    # colour: h = relu(-0.5 + d_z) = 0.5; y = (0.5, -0.5, 0)
    dec_c = ([[0.0], [0.0], [0.0], [0.0], [1.0]], [-0.5], [[1.0, -1.0, 0.0]], [0.0, 0.0, 0.0])
    # scale: h = relu(-1) = 0 -> y = b2 = 0 -> ratio 1/2, clamped to 1 - |O| = 0.4
    dec_s = ([[1.0], [1.0], [1.0], [1.0], [1.0]], [-10.0], [[3.0, 3.0, 3.0]], [0.0, 0.0, 0.0])
    # quaternion: h = relu(delta) = 2 -> y = 2 (1, 0, 0, 0.5) + (0, 0, 0, 0) = (2, 0, 0, 1)
    dec_q = ([[0.0], [1.0], [0.0], [0.0], [0.0]], [0.0], [[1.0, 0.0, 0.0, 0.5]], [0.0, 0.0, 0.0, 0.0])
    w = pack([dec_o, dec_c, dec_s, dec_q])
    e = oracle.decode(one_cell(), dict(F=1, H=1, weights=w), axis_cam(), raw=True)
    np.testing.assert_array_equal(e["raw"][0], np.float32([0.5, 0.5, -0.5, 0.0, 0.0, 0.0, 0.0, 2.0, 0.0, 0.0, 1.0]))
    assert e["opacity64"][0] == pytest.approx(math.tanh(0.5), abs=1e-15)
    sig = lambda t: 1.0 / (1.0 + math.exp(-t))
    np.testing.assert_allclose(e["color64"][0], [sig(0.5), sig(-0.5), 0.5], atol=1e-15)
    np.testing.assert_allclose(e["scales"][0], np.float32([0.4 * 0.1, 0.4 * 0.2, 0.4 * 0.3]), rtol=2e-7)
    np.testing.assert_array_equal(e["rots"][0], np.float32([2, 0, 0, 1]))
    np.testing.assert_allclose(e["means"][0], [0.06, 0.0, 2.0], rtol=1e-7, atol=1e-9)


def test_mlp_matches_binary64_and_activations():
    """Raw outputs agree with a binary64 numpy evaluation of the same MLPs to
    binary32 accumulation error; the activations and the assembly agree with
    their definitions."""
    s, d = scenes.make_neural_scene(5, n_cells=300, K=6, F=16, H=24)
    cam = scenes.orbit_cameras(12, 640, 480)[3]
    e = oracle.decode(s, d, cam, raw=True)
    parts = unpack(d["weights"], 16, 24, 6)
    V = np.asarray(cam["viewmat"], np.float64)
    o = -V[:3, :3].T @ V[:3, 3]
    ex = s["cell_pos"].astype(np.float64) - o
    dist = np.linalg.norm(ex, axis=1)
    X = np.concatenate([s["features"].astype(np.float64), dist[:, None], ex / dist[:, None]], 1)
    ys = []
    for (W1, b1, W2, b2) in parts:
        h = np.maximum(0.0, X @ W1 + b1)
        y = h @ W2 + b2
        scale = np.maximum(1.0, np.abs(h) @ np.abs(W2) + np.abs(b2))
        ys.append((y, scale))
    raw = e["raw"].astype(np.float64)
    off = 0
    for (y, scale) in ys:
        w = y.shape[1]
        assert np.max(np.abs(raw[:, off:off + w] - y) / scale) < 2e-6
        off += w
    K = 6
    yo, yc, ysc, yq = np.split(raw, np.cumsum([K, 3 * K, 3 * K]), axis=1)
    np.testing.assert_allclose(e["opacity64"], np.tanh(yo).ravel(), atol=1e-15)
    np.testing.assert_allclose(e["color64"], (1 / (1 + np.exp(-yc))).reshape(-1, 3), atol=1e-15)
    np.testing.assert_array_equal(e["rots"], yq.reshape(-1, 4).astype(np.float32))
    ratio = np.minimum(1 / (1 + np.exp(-ysc.reshape(-1, 3))),
                       1 - np.linalg.norm(s["offsets"].astype(np.float64), axis=1)[:, None])
    np.testing.assert_allclose(e["scales"], np.maximum(ratio, 0) * np.repeat(s["cell_scale"], K, 0), rtol=2e-6)


def test_containment_of_decoded_gaussians():
    """Centres sit inside their cell at the offset's normalised position
    (R(Q)^T (mu - x) / S = O^pos) and every scale respects the clamp
    s <= (1 - |O^pos|) S; with a huge scale bias the clamp binds."""
    s, d = scenes.make_neural_scene(6, n_cells=400, K=5, F=8, H=8)
    cam = scenes.orbit_cameras(12, 320, 240)[0]
    K = 5
    for bias in (None, 50.0):
        w = d["weights"].copy()
        if bias is not None:
            parts = unpack(w, 8, 8, K)
            parts[2] = (parts[2][0], parts[2][1], parts[2][2], np.full_like(parts[2][3], bias))
            w = pack(parts)
        e = oracle.decode(s, dict(d, weights=w), cam)
        q = s["cell_rot"].astype(np.float64)
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        wq, xq, yq, zq = q.T
        R = np.stack([np.stack([1 - 2 * (yq * yq + zq * zq), 2 * (xq * yq - wq * zq), 2 * (xq * zq + wq * yq)], 1),
                      np.stack([2 * (xq * yq + wq * zq), 1 - 2 * (xq * xq + zq * zq), 2 * (yq * zq - wq * xq)], 1),
                      np.stack([2 * (xq * zq - wq * yq), 2 * (yq * zq + wq * xq), 1 - 2 * (xq * xq + yq * yq)], 1)], 1)
        Rg = np.repeat(R, K, 0)
        Sg = np.repeat(s["cell_scale"].astype(np.float64), K, 0)
        local = np.einsum("nji,nj->ni", Rg, e["means"] - np.repeat(s["cell_pos"], K, 0)) / Sg
        np.testing.assert_allclose(local, s["offsets"], atol=2e-4)
        lim = 1 - np.linalg.norm(s["offsets"].astype(np.float64), axis=1)
        assert (e["scales"] >= 0).all()
        assert (e["scales"] <= lim[:, None] * Sg * (1 + 1e-6) + 1e-12).all()
        if bias is not None:
            np.testing.assert_allclose(e["scales"], lim[:, None] * Sg, rtol=1e-6)


def test_decode_depends_on_camera_centre_only():
    """delta_n and d_n are the distance and world-space direction from the
    camera centre, so a rotated camera at the same centre decodes exactly the
    same Gaussians, and a moved one does not."""
    s, d = scenes.make_neural_scene(7, n_cells=200, K=4, F=8, H=8)
    eye = np.array([0.5, 2.0, 3.0])
    a = scenes.pinhole(scenes.look_at(eye, (0, 0, 0)), 320, 240)
    b = scenes.pinhole(scenes.look_at(eye, (1.0, 0.3, -0.5)), 320, 240)
    c = scenes.pinhole(scenes.look_at(eye + 0.1, (0, 0, 0)), 320, 240)
    ea, eb, ec = (oracle.decode(s, d, cam, raw=True) for cam in (a, b, c))
    assert np.abs(ea["raw"] - eb["raw"]).max() < 1e-5
    assert np.abs(ea["raw"] - ec["raw"]).max() > 1e-3
    np.testing.assert_array_equal(ea["means"], eb["means"])  # centres do not depend on the view at all


def test_zero_weights_give_activated_biases():
    """With zero matrices every output is its bias: opacity tanh(b),
    colour sigmoid(b), ratio sigmoid(b) (then clamped), quaternion b."""
    F, H, K = 4, 3, 2
    rng = np.random.default_rng(1)
    parts = []
    for a in A:
        parts.append((np.zeros((F + 4, H)), rng.normal(size=H), np.zeros((H, K * a)), rng.normal(size=K * a)))
    w = pack(parts)
    s, _ = scenes.make_neural_scene(2, n_cells=3, K=K, F=F, H=H)
    s["offsets"] = np.zeros_like(s["offsets"])
    e = oracle.decode(s, dict(F=F, H=H, weights=w), axis_cam())
    b = [np.float32(p[3]).astype(np.float64) for p in parts]
    np.testing.assert_allclose(e["opacity64"].reshape(3, K), np.tile(np.tanh(b[0]), (3, 1)), atol=1e-15)
    np.testing.assert_allclose(e["color64"].reshape(3, K * 3), np.tile(1 / (1 + np.exp(-b[1])), (3, 1)), atol=1e-15)
    ratio = 1 / (1 + np.exp(-b[2]))
    np.testing.assert_allclose(e["scales"].reshape(3, K * 3) / np.repeat(s["cell_scale"], K, 0).reshape(3, K * 3),
                               np.tile(ratio, (3, 1)), rtol=1e-6)
    np.testing.assert_array_equal(e["rots"].reshape(3, K * 4), np.tile(np.float32(b[3]), (3, 1)))
