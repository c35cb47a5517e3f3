"""CPU oracle of the Duplex-GS hybrid renderer (arXiv 2508.03180).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the renderer itself.  It shares no code
with the HIP library; the two meet only in the seeded inputs.

The arithmetic lives in ``duplex_oracle.c`` (plain C, binary64 for the
per-pixel recurrence, binary32 for the discrete cull/rectangle/depth
decisions).  This module builds it with gcc and marshals numpy arrays.

Parity status of each function (see the pins under tests/test_oracle_*.py):
  cells_discrete, gauss_discrete  pinned (brute-force rectangle checks,
                                  numerical-Jacobian projection, rigid motion)
  build_lists                     pinned (numpy stable sort, brute-force tiles)
  sh_basis                        pinned (scipy complex spherical harmonics)
  render (duplex, alpha, lcwsr)   pinned (K=1 -> sorted alpha blending,
                                  one cell -> weighted sum, permutation
                                  invariance, opaque front cell, hand-worked
                                  two-cell scene and its N^val / N^rendered
                                  counts, Gaussian mass, rigid motion, ragged
                                  cells -> the same scene padded to fixed K)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "duplex_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MAX_ALT = 8


def build(force=True):
    """Compile the C oracle into oracle/liboracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        alt = os.environ.get("DUPLEX_ORACLE_LIB")  # a mutated copy, for the mutation check
        if alt:
            path = alt
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            path = _LIB
        _lib = C.CDLL(path)
        _lib.orc_build_lists.restype = C.c_int64
        _lib.orc_render.restype = C.c_int64
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def camera_vector(cam):
    V = np.asarray(cam["viewmat"], np.float32)
    v = np.zeros(19, np.float32)
    v[0:9] = V[:3, :3].reshape(-1)
    v[9:12] = V[:3, 3]
    v[12:19] = [cam["fx"], cam["fy"], cam["cx"], cam["cy"], cam["width"], cam["height"], cam["z_near"]]
    return v


def num_threads():
    return int(_load().orc_num_threads())


def set_threads(n):
    """Threads the oracle's later calls use (timing of the CPU baseline)."""
    _load().orc_set_threads(C.c_int(int(n)))


def cells_discrete(scene, cam, kappa=1.0, delta=0.3):
    L = _load()
    N = scene["cell_pos"].shape[0]
    pos, sc, rot = _f32(scene["cell_pos"]), _f32(scene["cell_scale"]), _f32(scene["cell_rot"])
    vis = np.zeros(N, np.uint8)
    dep = np.zeros(N, np.uint32)
    rect = np.zeros((N, 4), np.int32)
    trect = np.zeros((N, 4), np.int32)
    nt = np.zeros(N, np.int32)
    L.orc_cells_discrete(C.c_int(N), _p(pos), _p(sc), _p(rot), _p(camera_vector(cam)), C.c_float(kappa),
                         C.c_float(delta), _p(vis), _p(dep), _p(rect), _p(trect), _p(nt))
    return dict(visible=vis, depth_bits=dep, rect=rect, trect=trect, ntiles=nt)


def gauss_discrete(scene, cam, delta=0.3):
    L = _load()
    M = scene["means"].shape[0]
    vis = np.zeros(M, np.uint8)
    dep = np.zeros(M, np.uint32)
    rect = np.zeros((M, 4), np.int32)
    nt = np.zeros(M, np.int32)
    L.orc_gauss_discrete(C.c_int(M), _p(_f32(scene["means"])), _p(_f32(scene["scales"])),
                         _p(_f32(scene["rots"])), _p(_f32(scene["opacities"])), _p(camera_vector(cam)),
                         C.c_float(delta), _p(vis), _p(dep), _p(rect), _p(nt))
    return dict(visible=vis, depth_bits=dep, rect=rect, ntiles=nt)


def build_lists(visible, depth_bits, rect, width, height):
    """Sorted (tile, depth, id) sequence: returns (ids, tiles, ranges[T,2])."""
    L = _load()
    P = int(visible.shape[0])
    vis = np.ascontiguousarray(visible, np.uint8)
    dep = np.ascontiguousarray(depth_bits, np.uint32)
    rect = np.ascontiguousarray(rect, np.int32)
    T = ((width + 15) // 16) * ((height + 15) // 16)
    ranges = np.zeros((T, 2), np.int32)
    cnt = L.orc_build_lists(C.c_int(P), _p(vis), _p(dep), _p(rect), C.c_int(width), C.c_int(height),
                            None, None, _p(ranges))
    ids = np.zeros(max(cnt, 1), np.int32)
    tiles = np.zeros(max(cnt, 1), np.int32)
    L.orc_build_lists(C.c_int(P), _p(vis), _p(dep), _p(rect), C.c_int(width), C.c_int(height),
                      _p(ids), _p(tiles), _p(ranges))
    return ids[:cnt], tiles[:cnt], ranges


DEFAULTS = dict(eps=1e-4, alpha_min=1.0 / 255.0, alpha_max=0.99, delta=0.3, kappa=1.0,
                bg=(0.0, 0.0, 0.0), v_one=False, no_et=False, band_alpha=1e-5, band_T=1e-4, tau=0.0)

MODES = {"duplex": 0, "alpha": 1, "lcwsr": 2}


def render(scene, cam, mode="duplex", pixels=None, alt_cap=None, **opts):
    """Render the whole image (pixels=None) or the listed (x, y) pixels.

    mode: "duplex" (the hybrid renderer), "alpha" (per-Gaussian sorted
    alpha blending) or "lcwsr" (the Duplex pipeline with LC-WSR cell weights
    v max(0, 1 - d / tau), tau > 0 given as an option).

    Returns a dict with color [P,3], D, T, last, nrend, nval, status
    (0 exact, 1 marginal, 2 unverifiable), n_alt, alt_slot and alt
    [slots, 8, 5] (C[3], D, T of each admissible alternative), n_keys.
    """
    o = dict(DEFAULTS)
    o.update(opts)
    L = _load()
    N = scene["cell_pos"].shape[0]
    offs = scene.get("cell_offsets")
    if offs is not None:  # variable members per cell (CSR)
        offs = np.ascontiguousarray(offs, np.int32)
        K, M = 0, int(offs[-1])
    else:
        K = int(scene["K"])
        M = N * K
    W, H = int(cam["width"]), int(cam["height"])
    if pixels is None:
        P = W * H
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, np.int32).reshape(-1, 2)
        P = pix.shape[0]
    ro = np.array([o["eps"], o["alpha_min"], o["alpha_max"], o["delta"], o["kappa"], o["bg"][0], o["bg"][1],
                   o["bg"][2], float(o["v_one"]), float(o["no_et"]), o["band_alpha"], o["band_T"], o["tau"]],
                  np.float64)
    if mode == "lcwsr" and not o["tau"] > 0:
        raise ValueError("the lcwsr mode needs tau > 0")
    color = np.zeros((P, 3), np.float64)
    D = np.zeros(P, np.float64)
    T = np.zeros(P, np.float64)
    last = np.zeros(P, np.int32)
    nrend = np.zeros(P, np.int32)
    nval = np.zeros(P, np.int32)
    status = np.zeros(P, np.int8)
    n_alt = np.zeros(P, np.int32)
    alt_slot = np.zeros(P, np.int32)
    if alt_cap is None:
        alt_cap = max(1024, P // 8)
    alt = np.zeros((alt_cap, MAX_ALT, 5), np.float64)
    alt_count = np.zeros(1, np.int32)
    nkeys = np.zeros(1, np.int32)
    sh = _f32(scene["sh"])
    vsh = _f32(scene["cell_v_sh"])
    cnt = L.orc_render(C.c_int(MODES[mode]), C.c_int(N), C.c_int(K), _p(offs), C.c_int(M),
                       _p(_f32(scene["cell_pos"])), _p(_f32(scene["cell_scale"])), _p(_f32(scene["cell_rot"])),
                       _p(vsh), C.c_int(int(scene["v_sh_degree"])), _p(_f32(scene["means"])),
                       _p(_f32(scene["scales"])), _p(_f32(scene["rots"])), _p(_f32(scene["opacities"])),
                       _p(sh), C.c_int(int(scene["sh_degree"])), _p(camera_vector(cam)), _p(ro), C.c_int(P),
                       _p(pix), _p(color), _p(D), _p(T), _p(last), _p(nrend), _p(nval), _p(status), _p(n_alt),
                       _p(alt_slot), _p(alt), C.c_int32(alt_cap), _p(alt_count), _p(nkeys))
    if cnt < 0:
        raise ValueError("cell_offsets must start at 0, never decrease and end at the number of Gaussians")
    return dict(color=color, D=D, T=T, last=last, nrend=nrend, nval=nval, status=status, n_alt=n_alt,
                alt_slot=alt_slot, alt=alt[:min(int(alt_count[0]), alt_cap)], n_keys=int(cnt))


def image(res, cam):
    """Planar [3,H,W] view of a whole-image result."""
    H, W = int(cam["height"]), int(cam["width"])
    return res["color"].reshape(H, W, 3).transpose(2, 0, 1)


def sh_basis(deg, dirs):
    L = _load()
    d = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Cn = (deg + 1) ** 2
    out = np.zeros((d.shape[0], Cn), np.float64)
    L.orc_sh_basis(C.c_int(deg), C.c_int(d.shape[0]), _p(d), _p(out))
    return out


def gauss_continuous(scene, cam, idx, delta=0.3):
    """Binary64 u (2), screen covariance xx,xy,yy (3, undilated), colour (3),
    conic of the dilated covariance (3) of the Gaussians in idx."""
    L = _load()
    idx = np.ascontiguousarray(idx, np.int32)
    out = np.zeros((idx.shape[0], 11), np.float64)
    L.orc_gauss_continuous(C.c_int(idx.shape[0]), _p(idx), _p(_f32(scene["means"])), _p(_f32(scene["scales"])),
                           _p(_f32(scene["rots"])), _p(_f32(scene["opacities"])), _p(_f32(scene["sh"])),
                           C.c_int(int(scene["sh_degree"])), _p(camera_vector(cam)), C.c_double(delta), _p(out))
    return out


def cell_v(scene, cam, idx):
    L = _load()
    idx = np.ascontiguousarray(idx, np.int32)
    out = np.zeros(idx.shape[0], np.float64)
    L.orc_cell_v(C.c_int(idx.shape[0]), _p(idx), _p(_f32(scene["cell_pos"])), _p(_f32(scene["cell_v_sh"])),
                 C.c_int(int(scene["v_sh_degree"])), _p(camera_vector(cam)), _p(out))
    return out


def admissible_max_err(gpu_color, res):
    """Per-pixel max-abs error of gpu_color [P,3] against the closest
    admissible oracle value.  Unverifiable pixels get NaN."""
    g = np.asarray(gpu_color, np.float64).reshape(-1, 3)
    err = np.abs(g - res["color"]).max(1)
    idx = np.nonzero(res["status"] == 1)[0]
    for i in idx:
        s = res["alt_slot"][i]
        if s < 0:
            continue
        for a in range(res["n_alt"][i]):
            err[i] = min(err[i], np.abs(g[i] - res["alt"][s, a, :3]).max())
    err[res["status"] == 2] = np.nan
    return err


# ------------------------------------------------------------- neural decode

DECODER_OUTPUTS = (1, 3, 3, 4)  # opacity, colour, scale ratio, quaternion (per Gaussian)


def decoder_size(F, H, K):
    return int(_load().orc_decoder_size(C.c_int(F), C.c_int(H), C.c_int(K)))


def exp32(x):
    """The binary32 exp of the decode (Cody-Waite + degree-7 Taylor)."""
    x = np.ascontiguousarray(x, np.float32).reshape(-1)
    out = np.zeros_like(x)
    _load().orc_exp32(C.c_int(x.size), _p(x), _p(out))
    return out


def decode(scene, decoder, cam, raw=False):
    """Decode the Gaussians of a neural scene for a camera (Sec. III-A,
    Sec. IV-A): returns an explicit scene (cells kept; means, scales and raw
    quaternions in binary32; opacity tanh(y) and colour sigmoid(y) rounded
    to binary32, colour as SH degree 0) plus the binary64 opacity/colour and,
    with raw=True, the raw decoder outputs [N, sum K a].

    scene: cell_pos [N,3], cell_scale, cell_rot, cell_v_sh, v_sh_degree, K,
    features [N,F], offsets [N*K,3]; decoder: dict(F, H, weights) with the
    packed float32 weights (see orc_decode)."""
    L = _load()
    N = scene["cell_pos"].shape[0]
    K = int(scene["K"])
    F, H = int(decoder["F"]), int(decoder["H"])
    w = _f32(decoder["weights"]).reshape(-1)
    assert w.size == decoder_size(F, H, K), "decoder weights have the wrong size"
    feat = _f32(scene["features"]).reshape(N, F)
    offs = _f32(scene["offsets"]).reshape(N * K, 3)
    M = N * K
    means = np.zeros((M, 3), np.float32)
    scales = np.zeros((M, 3), np.float32)
    rots = np.zeros((M, 4), np.float32)
    opac = np.zeros(M, np.float64)
    col = np.zeros((M, 3), np.float64)
    ysz = K * sum(DECODER_OUTPUTS)
    rawv = np.zeros((N, ysz), np.float32) if raw else None
    rc = L.orc_decode(C.c_int(N), C.c_int(K), C.c_int(F), C.c_int(H), _p(_f32(scene["cell_pos"])),
                      _p(_f32(scene["cell_scale"])), _p(_f32(scene["cell_rot"])), _p(feat), _p(offs), _p(w),
                      _p(camera_vector(cam)), _p(means), _p(scales), _p(rots), _p(opac), _p(col),
                      _p(rawv) if raw else None)
    if rc != 0:
        raise RuntimeError("orc_decode failed")
    y00 = 1.0 / (2.0 * np.sqrt(np.pi))
    out = {k: scene[k] for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "v_sh_degree", "K")}
    out.update(means=means, scales=scales, rots=rots, opacities=opac.astype(np.float32),
               sh=((col - 0.5) / y00).astype(np.float32).reshape(M, 1, 3), sh_degree=0,
               opacity64=opac, color64=col)
    if raw:
        out["raw"] = rawv
    return out
