"""Seeded synthetic scenes and cameras.

This module only draws inputs: cell proxies, their member Gaussians and
pinhole cameras.  It holds none of the renderer's arithmetic (no projection,
no blending, no spherical-harmonic evaluation), so the CPU oracle and the HIP
path can both consume its output without sharing any code.

Layout of a scene (all numpy, natural row-per-primitive order):

    cell_pos   [N,3]  f32   cell centre x_n                     (Sec. IV-A)
    cell_scale [N,3]  f32   cell semi-axes S_n (> 0)
    cell_rot   [N,4]  f32   cell quaternion Q_n, (w, x, y, z)
    cell_v_sh  [N,Cv] f32   SH coefficients of the logit of v_n  (Sec. V-A)
    means      [M,3]  f32   Gaussian centres mu, M = N*K, cell-contiguous
    scales     [M,3]  f32
    rots       [M,4]  f32   (w, x, y, z)
    opacities  [M]    f32   sigma in [0, 1]; <= 0 marks an invalid Gaussian
    sh         [M,C,3] f32  colour SH, C = (deg+1)^2

Member k of cell n is Gaussian n*K + k.

A camera is a dict with ``viewmat`` (world -> camera, row-major 4x4, OpenCV
axes: x right, y down, z forward), ``fx, fy, cx, cy``, ``width, height`` and
``z_near``.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial.transform import Rotation

# Degree-0 real SH constant 1/(2*sqrt(pi)); used only to encode a chosen RGB
# into a DC coefficient so that a degree-0 scene renders that RGB.
_Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _points_in_unit_ball(rng, n):
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.random(n) ** (1.0 / 3.0)
    return d * r[:, None]


def _rotate(q_wxyz, v):
    """Rotate vectors v[i] by quaternions q[i] with scipy (scalar-last API)."""
    return Rotation.from_quat(q_wxyz[:, [1, 2, 3, 0]]).apply(v)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _members(rng, cell_pos, cell_scale, cell_rot, K, log_s_mu, log_s_sd):
    """K Gaussians per cell with centres uniform inside the cell ellipsoid."""
    N = cell_pos.shape[0]
    u = _points_in_unit_ball(rng, N * K)
    rep = np.repeat(np.arange(N), K)
    off = _rotate(cell_rot[rep].astype(np.float64), u * cell_scale[rep])
    means = cell_pos[rep] + off
    scales = np.exp(rng.normal(log_s_mu, log_s_sd, (N * K, 3)))
    rots = _unit_quats(rng, N * K)
    return means, scales, rots


def _v_sh(rng, N, degree=1):
    """Logit-SH of the calibration scalar v_n: DC term gives a logit near 2."""
    C = (degree + 1) ** 2
    v = rng.normal(0.0, 0.3, (N, C))
    v[:, 0] = rng.normal(7.0, 1.75, N)  # x Y00 ~= logit 2.0 +- 0.5
    return v


def _f32(scene):
    out = {}
    for k, v in scene.items():
        out[k] = v.astype(np.float32) if isinstance(v, np.ndarray) and v.dtype.kind == "f" else v
    return out


def make_tiny_scene(seed=0, n_cells=2000, K=8):
    """2,000 cells x 8 Gaussians in [-1,1]^3, SH degree 0 (RGB uniform)."""
    rng = np.random.default_rng(seed)
    N = n_cells
    cell_pos = rng.uniform(-1.0, 1.0, (N, 3))
    cell_scale = np.exp(rng.normal(-3.0, 0.3, (N, 3)))
    cell_rot = _unit_quats(rng, N)
    cell_v_sh = _v_sh(rng, N, 1)
    means, scales, rots = _members(rng, cell_pos, cell_scale, cell_rot, K, -4.5, 0.4)
    opac = _sigmoid(rng.standard_normal(N * K))
    rgb = rng.uniform(0.0, 1.0, (N * K, 3))
    sh = ((rgb - 0.5) / _Y00)[:, None, :]
    return _f32(dict(cell_pos=cell_pos, cell_scale=cell_scale, cell_rot=cell_rot,
                     cell_v_sh=cell_v_sh, v_sh_degree=1, means=means, scales=scales,
                     rots=rots, opacities=opac, sh=sh, sh_degree=0, K=K))


def _clustered_centres(rng, N, n_clusters=50, bg_frac=0.10, bg_half=1.5):
    n_bg = int(round(N * bg_frac))
    n_cl = N - n_bg
    w = rng.dirichlet(np.ones(n_clusters))
    counts = rng.multinomial(n_cl, w)
    cmeans = rng.uniform(-1.0, 1.0, (n_clusters, 3))
    crot = _unit_quats(rng, n_clusters)
    cstd = np.exp(rng.uniform(math.log(0.03), math.log(0.3), (n_clusters, 3)))
    pts = []
    for c in range(n_clusters):
        if counts[c] == 0:
            continue
        local = rng.standard_normal((counts[c], 3)) * cstd[c]
        pts.append(cmeans[c] + _rotate(np.repeat(crot[c:c + 1], counts[c], 0), local))
    pts.append(rng.uniform(-bg_half, bg_half, (n_bg, 3)))
    pts = np.concatenate(pts, 0)
    return pts[rng.permutation(N)]


def make_mid_scene(seed=1, n_cells=100_000, K=10, sh_degree=3):
    """1M-Gaussian clustered scene: 50 anisotropic clusters + 10% background."""
    rng = np.random.default_rng(seed)
    N = n_cells
    cell_pos = _clustered_centres(rng, N)
    cell_scale = np.exp(rng.normal(-4.0, 0.3, (N, 3)))
    cell_rot = _unit_quats(rng, N)
    cell_v_sh = _v_sh(rng, N, 1)
    means, scales, rots = _members(rng, cell_pos, cell_scale, cell_rot, K, -5.5, 0.4)
    opac = _sigmoid(rng.normal(1.5, 1.5, N * K))
    C = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, (N * K, C, 3))
    return _f32(dict(cell_pos=cell_pos, cell_scale=cell_scale, cell_rot=cell_rot,
                     cell_v_sh=cell_v_sh, v_sh_degree=1, means=means, scales=scales,
                     rots=rots, opacities=opac, sh=sh, sh_degree=sh_degree, K=K))


def make_large_scene(seed=2, n_cells=600_000, K=10, sh_degree=3, extent=100.0,
                     height_mean=3.0, height_cut=20.0):
    """Ground-biased aerial-scale scene with radii spread over three decades."""
    rng = np.random.default_rng(seed)
    N = n_cells
    xz = rng.uniform(-extent, extent, (N, 2))
    # truncated exponential heights (inverse CDF)
    u = rng.random(N)
    y = -height_mean * np.log(1.0 - u * (1.0 - math.exp(-height_cut / height_mean)))
    cell_pos = np.stack([xz[:, 0], y, xz[:, 1]], 1)
    r = np.exp(rng.uniform(math.log(0.005), math.log(5.0), N))
    cell_scale = r[:, None] * np.exp(rng.normal(0.0, 0.3, (N, 3)))
    cell_rot = _unit_quats(rng, N)
    cell_v_sh = _v_sh(rng, N, 1)
    u = _points_in_unit_ball(rng, N * K)
    rep = np.repeat(np.arange(N), K)
    means = cell_pos[rep] + _rotate(cell_rot[rep], u * cell_scale[rep])
    scales = r[rep][:, None] * np.exp(rng.normal(-1.5, 0.4, (N * K, 3)))
    rots = _unit_quats(rng, N * K)
    opac = _sigmoid(rng.normal(1.5, 1.5, N * K))
    C = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.2, (N * K, C, 3))
    return _f32(dict(cell_pos=cell_pos, cell_scale=cell_scale, cell_rot=cell_rot,
                     cell_v_sh=cell_v_sh, v_sh_degree=1, means=means, scales=scales,
                     rots=rots, opacities=opac, sh=sh, sh_degree=sh_degree, K=K))


def make_neural_scene(seed=1, n_cells=100_000, K=10, F=32, H=32):
    """Cells of the clustered generator with a latent feature each and K
    offsets in the unit ball (|O^pos| <= 0.9), plus random decoder weights
    (no trained ones exist): N(0, 1/fan-in) matrices; biases set so that
    most Gaussians are valid (opacity logit +1.5), colours are mid-grey on
    average and scale ratios sit near 0.22 (member scale / cell scale of the
    explicit generator).  Returns (scene, decoder)."""
    rng = np.random.default_rng(seed)
    N = n_cells
    cell_pos = _clustered_centres(rng, N)
    cell_scale = np.exp(rng.normal(-4.0, 0.3, (N, 3)))
    cell_rot = _unit_quats(rng, N)
    cell_v_sh = _v_sh(rng, N, 1)
    feats = rng.normal(0.0, 1.0, (N, F))
    offs = _points_in_unit_ball(rng, N * K) * 0.9
    parts = []
    for a, bias in zip((1, 3, 3, 4), (1.5, 0.0, -1.25, None)):
        I, O = F + 4, K * a
        W1 = rng.normal(0.0, 1.0 / math.sqrt(I), (I, H))
        b1 = rng.normal(0.0, 0.1, H)
        W2 = rng.normal(0.0, 0.5 / math.sqrt(H), (H, O))
        if bias is None:  # quaternions: identity plus noise
            b2 = np.tile([2.0, 0.0, 0.0, 0.0], K) + rng.normal(0.0, 0.3, O)
        else:
            b2 = bias + rng.normal(0.0, 0.3, O)
        parts += [W1.ravel(), b1, W2.ravel(), b2]
    scene = _f32(dict(cell_pos=cell_pos, cell_scale=cell_scale, cell_rot=cell_rot, cell_v_sh=cell_v_sh,
                      v_sh_degree=1, K=K, features=feats, offsets=offs))
    decoder = dict(F=F, H=H, weights=np.concatenate(parts).astype(np.float32))
    return scene, decoder


def make_ragged_scene(seed=0, n_cells=1500, k_max=32, sh_degree=0):
    """Tiny-scene cells that each emit their own number of Gaussians (Sec.
    IV-A: a cell spawns its Gaussians; nothing fixes their count): counts
    uniform over 0..k_max with a tenth of the cells at k_max and a twentieth
    empty, stored as CSR offsets ``cell_offsets`` [N+1] (members of cell n
    are Gaussians cell_offsets[n] .. cell_offsets[n+1]-1)."""
    rng = np.random.default_rng(seed)
    N = n_cells
    counts = rng.integers(0, k_max + 1, N)
    counts[rng.random(N) < 0.1] = k_max
    counts[rng.random(N) < 0.05] = 0
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    M = int(offsets[-1])
    cell_pos = rng.uniform(-1.0, 1.0, (N, 3))
    cell_scale = np.exp(rng.normal(-3.0, 0.3, (N, 3)))
    cell_rot = _unit_quats(rng, N)
    cell_v_sh = _v_sh(rng, N, 1)
    rep = np.repeat(np.arange(N), counts)
    u = _points_in_unit_ball(rng, M)
    means = cell_pos[rep] + _rotate(cell_rot[rep].astype(np.float64), u * cell_scale[rep])
    scales = np.exp(rng.normal(-4.5, 0.4, (M, 3)))
    rots = _unit_quats(rng, M)
    opac = _sigmoid(rng.standard_normal(M))
    C = (sh_degree + 1) ** 2
    sh = np.concatenate([((rng.uniform(0.0, 1.0, (M, 3)) - 0.5) / _Y00)[:, None, :],
                         rng.normal(0.0, 0.2, (M, C - 1, 3))], 1)
    out = _f32(dict(cell_pos=cell_pos, cell_scale=cell_scale, cell_rot=cell_rot, cell_v_sh=cell_v_sh,
                    v_sh_degree=1, means=means, scales=scales, rots=rots, opacities=opac, sh=sh,
                    sh_degree=sh_degree, K=k_max))
    out["cell_offsets"] = offsets
    return out


def pad_to_fixed_k(scene, K=None):
    """The same scene with K members per cell: each cell's Gaussians in their
    order, then invalid ones (opacity 0) up to K.  Renders identically (an
    invalid Gaussian has no keys and no contribution)."""
    offs = np.asarray(scene["cell_offsets"], np.int64)
    counts = np.diff(offs)
    N = counts.shape[0]
    K = int(counts.max()) if K is None else K
    slot = np.arange(K)[None, :]
    have = slot < counts[:, None]
    src = np.where(have, offs[:-1, None] + slot, 0).reshape(-1)
    out = {k: v for k, v in scene.items() if k != "cell_offsets"}
    for k in ("means", "scales", "rots", "sh"):
        out[k] = np.ascontiguousarray(scene[k][src])
    out["opacities"] = np.where(have.reshape(-1), scene["opacities"][src], 0.0).astype(np.float32)
    out["K"] = K
    assert N == scene["cell_pos"].shape[0]
    return out


def subset_scene(scene, cells):
    """Scene restricted to the given cell indices (members follow their cells)."""
    cells = np.asarray(cells)
    K = scene["K"]
    g = (cells[:, None] * K + np.arange(K)[None, :]).reshape(-1)
    out = dict(scene)
    for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh"):
        out[k] = np.ascontiguousarray(scene[k][cells])
    for k in ("means", "scales", "rots", "opacities", "sh"):
        out[k] = np.ascontiguousarray(scene[k][g])
    return out


# ----------------------------------------------------------------- cameras

def look_at(eye, target, up=(0.0, 1.0, 0.0)):
    """World->camera 4x4 with OpenCV axes (x right, y down, z forward)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(r) < 1e-6:  # looking along `up`: pick another reference
        r = np.cross(f, np.array([0.0, 0.0, 1.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    Rm = np.stack([r, d, f], 0)
    V = np.eye(4)
    V[:3, :3] = Rm
    V[:3, 3] = -Rm @ eye
    return V.astype(np.float32)


def pinhole(viewmat, width, height, fov_x_deg=60.0, z_near=0.2):
    f = 0.5 * width / math.tan(math.radians(fov_x_deg) * 0.5)
    return dict(viewmat=np.asarray(viewmat, np.float32), fx=float(f), fy=float(f),
                cx=0.5 * width, cy=0.5 * height, width=int(width), height=int(height),
                z_near=float(z_near))


def tiny_camera(width=256, height=256):
    el, az = math.radians(20.0), math.radians(30.0)
    eye = 3.0 * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return pinhole(look_at(eye, (0, 0, 0)), width, height)


def orbit_cameras(n_frames=60, width=1920, height=1080, radius=3.0, elevation_deg=15.0,
                  step_deg=6.0, fov_x_deg=60.0):
    el = math.radians(elevation_deg)
    cams = []
    for i in range(n_frames):
        az = math.radians(step_deg * i)
        eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
        cams.append(pinhole(look_at(eye, (0, 0, 0)), width, height, fov_x_deg))
    return cams


def aerial_orbit_cameras(n_frames=60, width=1920, height=1080, radius=120.0, altitude=80.0, step_deg=6.0,
                         fov_x_deg=60.0):
    """Orbit above the large scene, looking at the origin."""
    cams = []
    for i in range(n_frames):
        az = math.radians(step_deg * i)
        eye = np.array([radius * math.sin(az), altitude, radius * math.cos(az)])
        cams.append(pinhole(look_at(eye, (0, 0, 0)), width, height, fov_x_deg))
    return cams


def large_scene_cameras(seed=2, width=1280, height=720, n_near=20, n_far=20, extent=100.0):
    """Near (street-level) and far (aerial) views of the large scene."""
    rng = np.random.default_rng(seed + 1000)
    cams = []
    for _ in range(n_near):
        h = rng.uniform(1.5, 10.0)
        pos = np.array([rng.uniform(-0.8 * extent, 0.8 * extent), h,
                        rng.uniform(-0.8 * extent, 0.8 * extent)])
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-20.0, 5.0))
        d = np.array([math.cos(pitch) * math.sin(yaw), math.sin(pitch), math.cos(pitch) * math.cos(yaw)])
        cams.append(pinhole(look_at(pos, pos + d), width, height))
    for _ in range(n_far):
        h = rng.uniform(60.0, 150.0)
        ang = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(0.0, 150.0)
        pos = np.array([rad * math.cos(ang), h, rad * math.sin(ang)])
        tgt = np.array([rng.uniform(-0.5 * extent, 0.5 * extent), 0.0,
                        rng.uniform(-0.5 * extent, 0.5 * extent)])
        cams.append(pinhole(look_at(pos, tgt), width, height))
    return cams
