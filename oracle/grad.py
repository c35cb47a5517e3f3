"""Binary64 gradient oracle of the Duplex-GS hybrid renderer (PyTorch, CPU).

TEST INFRASTRUCTURE ONLY (used by the test-suite), independent of the HIP
library.  It evaluates the dense formulation of the hybrid renderer
(Sec. V-A, eq. hybrid_renderer with w_n = v_n T_n, eq. dulpex_T; cell-level
termination, Sec. V-B; box skip, Sec. VI-A) as differentiable binary64
tensor code, with every discrete choice frozen: the pixel boxes and tile
lists come from the C oracle's binary32 discrete layer, and the alpha_min and
termination gates are taken on the binary64 values without gradient.  The
loss gradient then comes from autograd.

Pins: its forward equals the C oracle's per pixel (tests), and its autograd
gradient equals central finite differences of its own forward (tests).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import DEFAULTS, build_lists, cells_discrete, gauss_discrete

PI = math.pi


def sh_basis(deg, d):
    """Real SH (Condon-Shortley phase, m = -l..l) of unit directions d [n,3]."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    cols = [torch.full_like(x, 0.5 * math.sqrt(1 / PI))]
    if deg >= 1:
        c1 = math.sqrt(3 / (4 * PI))
        cols += [-c1 * y, c1 * z, -c1 * x]
    if deg >= 2:
        xx, yy, zz = x * x, y * y, z * z
        cols += [0.5 * math.sqrt(15 / PI) * x * y, -0.5 * math.sqrt(15 / PI) * y * z,
                 0.25 * math.sqrt(5 / PI) * (2 * zz - xx - yy), -0.5 * math.sqrt(15 / PI) * x * z,
                 0.25 * math.sqrt(15 / PI) * (xx - yy)]
    if deg >= 3:
        cols += [-0.125 * math.sqrt(70 / PI) * y * (3 * xx - yy), 0.5 * math.sqrt(105 / PI) * x * y * z,
                 -0.125 * math.sqrt(42 / PI) * y * (4 * zz - xx - yy),
                 0.25 * math.sqrt(7 / PI) * z * (2 * zz - 3 * xx - 3 * yy),
                 -0.125 * math.sqrt(42 / PI) * x * (4 * zz - xx - yy), 0.25 * math.sqrt(105 / PI) * z * (xx - yy),
                 -0.125 * math.sqrt(70 / PI) * x * (xx - 3 * yy)]
    return torch.stack(cols, 1)


def quat_to_rot(q):
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)


def _camera(cam):
    V = torch.tensor(np.asarray(cam["viewmat"], np.float32).astype(np.float64))
    f = {k: float(np.float32(cam[k])) for k in ("fx", "fy", "cx", "cy")}
    return V[:3, :3], V[:3, 3], f


def project(means, scales, rots, cam, delta):
    """Projected means u [n,2] and conics (A, B, C) of the dilated screen
    covariance (EWA: Jacobian of the perspective map at the centre with the
    1.3 x half-FOV clamp)."""
    Rc, tc, f = _camera(cam)
    t = means @ Rc.T + tc
    tx, ty, tz = t.unbind(1)
    u = torch.stack([f["fx"] * tx / tz + f["cx"], f["fy"] * ty / tz + f["cy"]], 1)
    limx = 1.3 * (0.5 * cam["width"] / f["fx"])
    limy = 1.3 * (0.5 * cam["height"] / f["fy"])
    xr = torch.clamp(tx / tz, -limx, limx)
    yr = torch.clamp(ty / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([f["fx"] / tz, zero, -f["fx"] * xr / tz], 1),
                     torch.stack([zero, f["fy"] / tz, -f["fy"] * yr / tz], 1)], 1)
    R = quat_to_rot(rots)
    S = R * scales[:, None, :]
    Sig = S @ S.transpose(1, 2)
    Mx = J @ Rc
    cov = Mx @ Sig @ Mx.transpose(1, 2)
    a = cov[:, 0, 0] + delta
    b = 0.5 * (cov[:, 0, 1] + cov[:, 1, 0])
    c = cov[:, 1, 1] + delta
    det = a * c - b * b
    return u, torch.stack([c / det, -b / det, a / det], 1)


def unit_dirs(points, cam):
    Rc, tc, _ = _camera(cam)
    o = -Rc.T @ tc
    d = points - o
    return d / d.norm(dim=1, keepdim=True)


class FrozenScene:
    """Discrete decisions of one (scene, camera, options) from the C oracle."""

    def __init__(self, scene, cam, kappa=1.0, delta=0.3):
        self.cam = cam
        N = scene["cell_pos"].shape[0]
        offs = scene.get("cell_offsets")
        # members of cell n: Gaussians first[n] .. first[n + 1] - 1
        self.first = (np.asarray(offs, np.int64) if offs is not None
                      else np.arange(N + 1, dtype=np.int64) * int(scene["K"]))
        counts = np.diff(self.first)
        self.K = int(counts.max()) if N else 1
        self.cd = cells_discrete(scene, cam, kappa, delta)
        self.gd = gauss_discrete(scene, cam, delta)
        W, H = int(cam["width"]), int(cam["height"])
        self.ids, _, self.ranges = build_lists(self.cd["visible"], self.cd["depth_bits"], self.cd["rect"], W, H)


def render(params, frozen: FrozenScene, pixels, return_masks=False, **opts):
    """Differentiable render of the listed (x, y) pixels.

    params: dict of float64 tensors cell_pos [N,3], cell_v_sh [N,Cv], means
    [M,3], scales [M,3], rots [M,4], opacities [M], sh [M,C,3] (any may
    require grad).  Returns colour [P,3], D [P], T [P]."""
    o = dict(DEFAULTS)
    o.update(opts)
    cam, K = frozen.cam, frozen.K
    W = int(cam["width"])
    TX = (W + 15) // 16
    pix = np.asarray(pixels, np.int64).reshape(-1, 2)
    P = pix.shape[0]
    # per-pixel frozen tile lists
    tiles = (pix[:, 1] // 16) * TX + pix[:, 0] // 16
    lens = frozen.ranges[tiles, 1] - frozen.ranges[tiles, 0]
    L = max(int(lens.max()) if P else 0, 1)
    CI = np.full((P, L), -1, np.int64)
    for i in range(P):
        s, e = frozen.ranges[tiles[i]]
        CI[i, :e - s] = frozen.ids[s:e]
    valid = CI >= 0
    cell = np.where(valid, CI, 0)
    kk = np.arange(max(K, 1))[None, None, :]
    member = valid[:, :, None] & (kk < np.diff(frozen.first)[cell][:, :, None])
    G = np.where(member, frozen.first[cell][:, :, None] + kk, 0)
    rect = frozen.gd["rect"][G]
    inbox = (member & frozen.gd["visible"][G].astype(bool)
             & (pix[:, None, None, 0] >= rect[..., 0]) & (pix[:, None, None, 0] <= rect[..., 1])
             & (pix[:, None, None, 1] >= rect[..., 2]) & (pix[:, None, None, 1] <= rect[..., 3]))
    # continuous quantities
    # the dilation is a binary32 option on both sides of the comparison
    u, con = project(params["means"], params["scales"], params["rots"], cam, float(np.float32(o["delta"])))
    deg = round(params["sh"].shape[1] ** 0.5) - 1
    Y = sh_basis(deg, unit_dirs(params["means"], cam))
    col = torch.clamp(0.5 + torch.einsum("mc,mcd->md", Y, params["sh"]), min=0.0)
    if o["v_one"]:
        v = torch.ones(params["cell_pos"].shape[0], dtype=torch.float64)
    else:
        vdeg = round(params["cell_v_sh"].shape[1] ** 0.5) - 1
        Yv = sh_basis(vdeg, unit_dirs(params["cell_pos"], cam))
        v = torch.sigmoid((Yv * params["cell_v_sh"]).sum(1))
    Gt = torch.from_numpy(G)
    q = torch.from_numpy(pix).to(torch.float64) + 0.5
    dx = q[:, None, None, 0] - u[Gt, 0]
    dy = q[:, None, None, 1] - u[Gt, 1]
    cg = con[Gt]
    power = -0.5 * (cg[..., 0] * dx * dx + 2 * cg[..., 1] * dx * dy + cg[..., 2] * dy * dy)
    alpha = torch.clamp(params["opacities"][Gt] * torch.exp(power), max=o["alpha_max"])
    gate = torch.from_numpy(inbox) & (alpha.detach() >= o["alpha_min"])
    a = torch.where(gate, alpha, torch.zeros_like(alpha))
    vc = v[torch.from_numpy(cell)]
    A = (a[..., None] * col[Gt]).sum(2)
    B = a.sum(2)
    Pc = torch.prod(1 - vc[..., None] * a, 2)
    Tb = torch.cat([torch.ones(P, 1, dtype=torch.float64), torch.cumprod(Pc, 1)[:, :-1]], 1)
    eps = 0.0 if o["no_et"] else o["eps"]
    inc = torch.from_numpy(valid) & (Tb.detach() >= eps)
    w = torch.where(inc, vc * Tb, torch.zeros_like(Tb))
    N = (w[..., None] * A).sum(1)
    D = (w * B).sum(1)
    bg = torch.tensor(o["bg"], dtype=torch.float64)
    C = torch.where((D > 0)[:, None], N / torch.where(D > 0, D, torch.ones_like(D))[:, None], bg[None, :])
    T = torch.where(inc, Pc, torch.ones_like(Pc)).prod(1)
    if return_masks:
        return C, D, T, (gate, inc)
    return C, D, T


def params_from_scene(scene, requires_grad=True):
    keys = ("cell_pos", "cell_v_sh", "means", "scales", "rots", "opacities", "sh")
    return {k: torch.tensor(np.asarray(scene[k], np.float32).astype(np.float64), requires_grad=requires_grad)
            for k in keys}


def gradients(scene, cam, pixels, grad_color, grad_D=None, **opts):
    """Gradient of L = sum grad_color . C + sum grad_D D over the pixels."""
    fz = FrozenScene(scene, cam, opts.get("kappa", 1.0), opts.get("delta", 0.3))
    p = params_from_scene(scene)
    C, D, _ = render(p, fz, pixels, **opts)
    L = (C * torch.as_tensor(grad_color, dtype=torch.float64)).sum()
    if grad_D is not None:
        L = L + (D * torch.as_tensor(grad_D, dtype=torch.float64)).sum()
    L.backward()
    return {k: (v.grad.numpy() if v.grad is not None else np.zeros(v.shape)) for k, v in p.items()}
