"""Torch-facing wrapper of the C ABI.

PyTorch only provides device memory and streams here: scenes are uploaded
once into planar device tensors, outputs are preallocated tensors, and every
step of a frame runs in the HIP library.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _capi as capi


def _planar(a, device):
    """[P, ...] numpy -> planar [..., P] contiguous float32 device tensor."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    t = torch.as_tensor(a.reshape(a.shape[0], int(np.prod(a.shape[1:], dtype=np.int64))))
    t = t.t().contiguous()
    return t.to(device)


def _planar_t(t):
    """[P, ...] torch tensor -> planar [..., P] contiguous float32."""
    return t.detach().reshape(t.shape[0], -1).t().contiguous().float()


class DeviceScene:
    """A scene resident in device memory in the library's planar layout.
    With tensors["cell_offsets"] (int32 [N+1]) the cells have their own
    member counts (at most K each) and M = offsets[N]."""

    def __init__(self, tensors, N, K, v_sh_degree, sh_degree, M=None):
        self.t = tensors
        self.N, self.K = int(N), int(K)
        self.M = self.N * self.K if M is None else int(M)
        self.v_sh_degree, self.sh_degree = int(v_sh_degree), int(sh_degree)

    @classmethod
    def from_numpy(cls, scene, device="cuda"):
        N = scene["cell_pos"].shape[0]
        K = int(scene["K"])
        sh = np.asarray(scene["sh"], np.float32)  # [M, C, 3] -> [C, 3, M]
        t = dict(cell_pos=_planar(scene["cell_pos"], device), cell_scale=_planar(scene["cell_scale"], device),
                 cell_rot=_planar(scene["cell_rot"], device), cell_v_sh=_planar(scene["cell_v_sh"], device),
                 means=_planar(scene["means"], device), scales=_planar(scene["scales"], device),
                 rots=_planar(scene["rots"], device),
                 opacities=torch.as_tensor(np.ascontiguousarray(scene["opacities"], np.float32)).to(device),
                 sh=torch.as_tensor(np.ascontiguousarray(sh.transpose(1, 2, 0))).to(device))
        M = None
        if scene.get("cell_offsets") is not None:
            offs = np.ascontiguousarray(scene["cell_offsets"], np.int32)
            t["cell_offsets"] = torch.as_tensor(offs).to(device)
            M = int(offs[-1])
        return cls(t, N, K, scene["v_sh_degree"], scene["sh_degree"], M)

    @classmethod
    def from_tensors(cls, cell_pos, cell_scale, cell_rot, cell_v_sh, means, scales, rots, opacities, sh, K):
        """From natural-layout device tensors ([N,3], [N,3], [N,4], [N,Cv],
        [M,3], [M,3], [M,4], [M], [M,C,3]); planar copies are made."""
        Cv, C = cell_v_sh.shape[1], sh.shape[1]
        t = dict(cell_pos=_planar_t(cell_pos), cell_scale=_planar_t(cell_scale), cell_rot=_planar_t(cell_rot),
                 cell_v_sh=_planar_t(cell_v_sh), means=_planar_t(means), scales=_planar_t(scales),
                 rots=_planar_t(rots), opacities=opacities.detach().contiguous().float(),
                 sh=sh.detach().permute(1, 2, 0).contiguous().float())
        return cls(t, cell_pos.shape[0], K, round(Cv ** 0.5) - 1, round(C ** 0.5) - 1)

    def nbytes(self):
        return sum(v.numel() * v.element_size() for v in self.t.values())

    def struct(self):
        s = capi.dgs_scene()
        s.num_cells = self.N
        s.gaussians_per_cell = self.K
        for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "means", "scales", "rots", "opacities", "sh"):
            setattr(s, k, self.t[k].data_ptr() if self.t[k].numel() else None)
        s.v_sh_degree = self.v_sh_degree
        s.sh_degree = self.sh_degree
        if "cell_offsets" in self.t:
            s.cell_offsets = self.t["cell_offsets"].data_ptr()
            s.num_gaussians = self.M
        return s


class NeuralDeviceScene:
    """Neural scene (cells + features + offsets) and its decoder weights in
    device memory, planar."""

    def __init__(self, tensors, N, K, v_sh_degree, F, H, weights):
        self.t, self.N, self.K, self.v_sh_degree = tensors, N, K, v_sh_degree
        self.F, self.H, self.weights = F, H, weights
        self.M = N * K

    @classmethod
    def from_numpy(cls, scene, decoder, device="cuda"):
        N, K = scene["cell_pos"].shape[0], int(scene["K"])
        t = {k: _planar(scene[k], device) for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "features",
                                                   "offsets")}
        w = torch.tensor(np.asarray(decoder["weights"], np.float32).reshape(-1), device=device)
        return cls(t, N, K, int(scene["v_sh_degree"]), int(decoder["F"]), int(decoder["H"]), w)

    def struct(self):
        s = capi.dgs_neural_scene()
        s.num_cells, s.gaussians_per_cell = self.N, self.K
        for k in ("cell_pos", "cell_scale", "cell_rot", "cell_v_sh", "features", "offsets"):
            setattr(s, k, self.t[k].data_ptr() if self.t[k].numel() else None)
        s.v_sh_degree = self.v_sh_degree
        return s

    def decoder_struct(self):
        return capi.dgs_decoder(self.F, self.H, self.weights.data_ptr())


def camera_struct(cam):
    c = capi.dgs_camera()
    V = np.asarray(cam["viewmat"], np.float32).reshape(-1)
    for i in range(16):
        c.viewmat[i] = float(V[i])
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.z_near = float(cam.get("z_near", 0.2))
    return c


MODES = {"duplex": capi.DGS_MODE_DUPLEX, "alpha": capi.DGS_MODE_ALPHA, "lcwsr": capi.DGS_MODE_LCWSR}


def opts_struct(mode="duplex", v_one=False, no_et=False, stats=False, eps=None, alpha_min=None, alpha_max=None,
                delta=None, kappa=None, bg=None, tau=None):
    o = capi.dgs_render_opts()
    capi.dgs_default_opts(o)
    o.mode = MODES[mode]
    if tau is not None:
        o.lcwsr_tau = tau
    o.flags = (capi.DGS_FLAG_V_ONE if v_one else 0) | (capi.DGS_FLAG_NO_ET if no_et else 0) | \
              (capi.DGS_FLAG_STATS if stats else 0)
    if eps is not None:
        o.eps_T = eps
    if alpha_min is not None:
        o.alpha_min = alpha_min
    if alpha_max is not None:
        o.alpha_max = alpha_max
    if delta is not None:
        o.cov2d_dilation = delta
    if kappa is not None:
        o.proxy_kappa = kappa
    if bg is not None:
        for i in range(3):
            o.bg[i] = float(bg[i])
    return o


class Frame:
    """A saved Duplex frame (the library's dgs_frame): what its backward
    replays, kept apart from later renders.  Released when closed or
    garbage-collected."""

    def __init__(self, renderer, handle):
        self.renderer, self.handle = renderer, handle

    def stats(self):
        s = capi.dgs_frame_stats(self.renderer.ctx, self.handle)
        return dict(num_keys=s.num_keys, n_val=s.n_val, n_rendered=s.n_rendered, n_box=s.n_box,
                    n_cell_hits=s.n_cell_hits, n_cell_pixels=s.n_cell_pixels)

    def release(self):
        r, self.renderer = self.renderer, None
        if r is not None and r.ctx and self.handle:
            capi.check(capi.dgs_frame_release(r.ctx, self.handle), r.ctx)
        self.handle = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Renderer:
    """One library context bound to a device and a stream.  overlap: run a
    Duplex frame's member projection on a second stream beside the cell sort
    (turn it off when several renderers already overlap whole frames)."""

    def __init__(self, device=0, stream=None, overlap=True):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = capi.dgs_create(self.device.index or 0, self.stream.cuda_stream)
        if not overlap:
            capi.dgs_set_overlap(self.ctx, False)

    def close(self):
        if self.ctx:
            capi.dgs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_keys, max_prims=0, max_tiles=0):
        capi.dgs_reserve(self.ctx, max_keys, max_prims, max_tiles)

    def alloc_image(self, cam, aux=True):
        H, W = int(cam["height"]), int(cam["width"])
        d = self.device
        out = dict(color=torch.empty((3, H, W), device=d, dtype=torch.float32))
        if aux:
            out.update(D=torch.empty((H, W), device=d, dtype=torch.float32),
                       T=torch.empty((H, W), device=d, dtype=torch.float32),
                       last=torch.empty((H, W), device=d, dtype=torch.int32))
        return out

    def render_into(self, scene: DeviceScene, cam, out, opts, saved=None):
        """Enqueue one frame (no host synchronisation); returns the status.
        saved: None, or a capi.dgs_frame() that receives a saved-frame handle."""
        img = capi.dgs_image()
        img.color = out["color"].data_ptr()
        img.weight_sum = out["D"].data_ptr() if "D" in out else None
        img.final_T = out["T"].data_ptr() if "T" in out else None
        img.last = out["last"].data_ptr() if "last" in out else None
        return capi.dgs_render(self.ctx, scene.struct(), camera_struct(cam), opts, img, saved)

    def render_backward(self, scene: DeviceScene, frame, grad_color, grad_D=None, mean2d=False, into=None):
        """Gradients (planar, float32) of a loss whose gradient w.r.t. the
        colour of the saved frame `frame` (a Frame from render(save=True)) is
        grad_color [3,H,W] (and w.r.t. D, grad_D).  Without `into`, new
        buffers are returned, written whole by the library; with `into` (a
        dict as returned here), the gradients are added to its buffers and it
        is returned."""
        d = self.device
        M, N = scene.M, scene.N
        if into is None:
            g = dict(means=torch.empty((3, M), device=d), scales=torch.empty((3, M), device=d),
                     rots=torch.empty((4, M), device=d), opacities=torch.empty((M,), device=d),
                     sh=torch.empty_like(scene.t["sh"]), cell_v_sh=torch.empty_like(scene.t["cell_v_sh"]),
                     cell_pos=torch.empty((3, N), device=d))
            if mean2d:
                g["mean2d"] = torch.empty((2, M), device=d)
        else:
            g = into
            if mean2d and "mean2d" not in g:
                raise ValueError("into has no mean2d buffer")
        gr = capi.dgs_grads()
        gr.overwrite = 1 if into is None else 0
        gr.d_means, gr.d_scales, gr.d_rots = g["means"].data_ptr(), g["scales"].data_ptr(), g["rots"].data_ptr()
        gr.d_opacities, gr.d_sh = g["opacities"].data_ptr(), g["sh"].data_ptr()
        gr.d_cell_v_sh, gr.d_cell_pos = g["cell_v_sh"].data_ptr(), g["cell_pos"].data_ptr()
        gr.d_mean2d = g["mean2d"].data_ptr() if "mean2d" in g and (mean2d or into is not None) else None
        gc = grad_color.contiguous().float()
        gd = grad_D.contiguous().float() if grad_D is not None else None
        st = capi.dgs_render_backward(self.ctx, scene.struct(), None, None, frame.handle, gc.data_ptr(),
                                      gd.data_ptr() if gd is not None else None, gr)
        capi.check(st, self.ctx)
        return g

    def render(self, scene: DeviceScene, cam, out=None, check=True, save=False, **kw):
        """Render a frame.  With check=True the call synchronises, and on a
        key-capacity overflow it reserves the reported count and renders
        again.  With save=True (Duplex) out["frame"] is a Frame whose
        backward can be taken later (render_backward)."""
        opts = opts_struct(**kw)
        if out is None:
            out = self.alloc_image(cam)

        def go():
            h = capi.dgs_frame() if save else None
            capi.check(self.render_into(scene, cam, out, opts, h), self.ctx)
            if save:
                out["frame"] = Frame(self, h)
        go()
        if check:
            st = capi.dgs_sync(self.ctx)
            if st == capi.DGS_ERR_CAPACITY:
                need = capi.dgs_get_stats(self.ctx).num_keys
                if save:
                    out.pop("frame").release()
                self.reserve(int(need * 1.25) + 4096)
                go()
                st = capi.dgs_sync(self.ctx)
            capi.check(st, self.ctx)
        return out

    def render_neural(self, scene: NeuralDeviceScene, cam, out=None, check=True, **kw):
        """Render a neural scene (decode of the visible cells, then the same
        pipeline); with check=True synchronises and retries on key-capacity
        overflow like render()."""
        opts = opts_struct(**kw)
        if out is None:
            out = self.alloc_image(cam)

        def go():
            img = capi.dgs_image(out["color"].data_ptr(), out["D"].data_ptr() if "D" in out else None,
                                 out["T"].data_ptr() if "T" in out else None,
                                 out["last"].data_ptr() if "last" in out else None)
            return capi.dgs_render_neural(self.ctx, scene.struct(), scene.decoder_struct(), camera_struct(cam), opts,
                                          img)
        capi.check(go(), self.ctx)
        if check:
            st = capi.dgs_sync(self.ctx)
            if st == capi.DGS_ERR_CAPACITY:
                self.reserve(int(capi.dgs_get_stats(self.ctx).num_keys * 1.25) + 4096)
                capi.check(go(), self.ctx)
                st = capi.dgs_sync(self.ctx)
            capi.check(st, self.ctx)
        return out

    def read_decoded(self, M):
        """Decoded Gaussians of the last neural render, row-major numpy-style
        tensors: means [M,3], scales [M,3], rots [M,4], opacities [M], colours [M,3]."""
        d = self.device
        t = dict(means=torch.empty((3, M), device=d), scales=torch.empty((3, M), device=d),
                 rots=torch.empty((4, M), device=d), opacities=torch.empty((M,), device=d),
                 colors=torch.empty((3, M), device=d))
        capi.dgs_read_decoded(self.ctx, t["means"].data_ptr(), t["scales"].data_ptr(), t["rots"].data_ptr(),
                              t["opacities"].data_ptr(), t["colors"].data_ptr())
        self.sync()
        return {k: (v.t().contiguous() if v.dim() == 2 else v) for k, v in t.items()}

    def sync(self):
        return capi.dgs_sync(self.ctx)

    def stats(self):
        s = capi.dgs_get_stats(self.ctx)
        return dict(num_keys=s.num_keys, key_capacity=s.key_capacity, n_val=s.n_val, n_rendered=s.n_rendered,
                    n_box=s.n_box, n_cell_hits=s.n_cell_hits, device_error=s.device_error,
                    sort_passes=s.sort_passes, n_cell_pixels=s.n_cell_pixels)

    def read_lists(self, tiles):
        n = self.stats()["num_keys"]
        keys = torch.empty(max(n, 1), dtype=torch.int64, device=self.device)
        vals = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        ranges = torch.empty((tiles, 2), dtype=torch.int32, device=self.device)
        capi.dgs_read_lists(self.ctx, keys.data_ptr(), vals.data_ptr(), ranges.data_ptr())
        self.stream.synchronize()
        return keys[:n], vals[:n], ranges

    def read_prims(self, P):
        rect = torch.empty((max(P, 1), 4), dtype=torch.int32, device=self.device)
        depth = torch.empty(max(P, 1), dtype=torch.int32, device=self.device)
        nt = torch.empty(max(P, 1), dtype=torch.int32, device=self.device)
        capi.dgs_read_prims(self.ctx, rect.data_ptr(), depth.data_ptr(), nt.data_ptr())
        self.stream.synchronize()
        return rect[:P], depth[:P], nt[:P]

    def read_gauss_rects(self, M):
        rect = torch.empty((max(M, 1), 4), dtype=torch.int32, device=self.device)
        capi.dgs_read_gauss_rects(self.ctx, rect.data_ptr())
        self.stream.synchronize()
        return rect[:M]

    def loss_l1_ssim(self, image, target, lam=0.2, grad=True):
        """(1 - lam) mean |image - target| + lam (1 - mean SSIM) of two
        contiguous float32 [C, H, W] device images, and dL/dimage when grad is
        set, computed by the library on the renderer's stream.  Returns
        (loss as a 0-dim tensor, gradient or None)."""
        if image.dtype != torch.float32 or target.dtype != torch.float32:
            raise ValueError("image and target must be float32")
        if image.dim() != 3 or image.shape != target.shape or not image.is_contiguous() or not target.is_contiguous():
            raise ValueError("image and target must be contiguous [C, H, W] tensors of one shape")
        C_, H, W = image.shape
        loss = torch.empty((), dtype=torch.float32, device=image.device)
        g = torch.empty_like(image) if grad else None
        capi.check(capi.dgs_loss_l1_ssim(self.ctx, image.data_ptr(), target.data_ptr(), C_, H, W, lam,
                                         loss.data_ptr(), g.data_ptr() if g is not None else 0), self.ctx)
        return loss, g

    def sort_pairs(self, keys, vals, key_bits):
        """In-place stable sort of int64 keys (as u64) and int32 values."""
        assert keys.dtype == torch.int64 and vals.dtype == torch.int32 and keys.is_contiguous()
        assert vals.is_contiguous() and keys.numel() == vals.numel()
        capi.dgs_sort_pairs(self.ctx, keys.data_ptr(), vals.data_ptr(), keys.numel(), key_bits)
        capi.check(capi.dgs_sync(self.ctx), self.ctx)


class DuplexRender(torch.autograd.Function):
    """Differentiable Duplex render through the C ABI.

    Inputs (natural layout, device): cell_pos [N,3], cell_scale [N,3],
    cell_rot [N,4], cell_v_sh [N,Cv], means [M,3], scales [M,3], rots [M,4],
    opacities [M], sh [M,C,3].  Returns (color [3,H,W], D [H,W]).  Cell
    scales and rotations only choose tiles, so their gradient is None.  The
    inputs are copied into the library's planar layout on every call; keep
    the parameters planar and use DuplexRenderPlanar to avoid that.  The
    frame is saved by the library, so any number of renders may await their
    backward on one Renderer.
    """

    @staticmethod
    def forward(ctx, renderer, cam, opts, cell_pos, cell_scale, cell_rot, cell_v_sh, means, scales, rots,
                opacities, sh):
        K = means.shape[0] // max(cell_pos.shape[0], 1)
        ds = DeviceScene.from_tensors(cell_pos, cell_scale, cell_rot, cell_v_sh, means, scales, rots, opacities,
                                      sh, K)
        out = renderer.render(ds, cam, mode="duplex", save=True, **opts)
        ctx.renderer, ctx.ds, ctx.frame = renderer, ds, out["frame"]
        ctx.shapes = (cell_v_sh.shape, sh.shape)
        ctx.hw = out["color"].shape[1:]
        return out["color"], out["D"]

    @staticmethod
    def backward(ctx, g_color, g_D):
        if g_color is None:
            g_color = torch.zeros((3, *ctx.hw), device=ctx.renderer.device)
        g = ctx.renderer.render_backward(ctx.ds, ctx.frame, g_color, g_D)
        cv_shape, sh_shape = ctx.shapes
        return (None, None, None, g["cell_pos"].t(), None, None, g["cell_v_sh"].t().reshape(cv_shape),
                g["means"].t(), g["scales"].t(), g["rots"].t(), g["opacities"], g["sh"].permute(2, 0, 1).reshape(sh_shape))


class DuplexRenderPlanar(torch.autograd.Function):
    """Differentiable Duplex render on parameters held in the library's
    planar layout (contiguous float32 device tensors, used in place with no
    copy): cell_pos [3,N], cell_scale [3,N], cell_rot [4,N], cell_v_sh [Cv,N],
    means [3,M], scales [3,M], rots [4,M], opacities [M], sh [C,3,M].  The
    gradients come back in the same layout, written whole by the library.
    Returns (color [3,H,W], D [H,W])."""

    @staticmethod
    def forward(ctx, renderer, cam, opts, cell_pos, cell_scale, cell_rot, cell_v_sh, means, scales, rots,
                opacities, sh):
        t = dict(cell_pos=cell_pos, cell_scale=cell_scale, cell_rot=cell_rot, cell_v_sh=cell_v_sh, means=means,
                 scales=scales, rots=rots, opacities=opacities, sh=sh)
        for k, v in t.items():
            if v.dtype != torch.float32 or not v.is_contiguous():
                raise ValueError(f"{k} must be a contiguous float32 tensor in the planar layout")
        N = cell_pos.shape[1]
        K = means.shape[1] // max(N, 1)
        ds = DeviceScene({k: v.detach() for k, v in t.items()}, N, K, round(cell_v_sh.shape[0] ** 0.5) - 1,
                         round(sh.shape[0] ** 0.5) - 1)
        out = renderer.render(ds, cam, mode="duplex", save=True, **opts)
        ctx.renderer, ctx.ds, ctx.frame = renderer, ds, out["frame"]
        ctx.hw = out["color"].shape[1:]
        return out["color"], out["D"]

    @staticmethod
    def backward(ctx, g_color, g_D):
        if g_color is None:
            g_color = torch.zeros((3, *ctx.hw), device=ctx.renderer.device)
        g = ctx.renderer.render_backward(ctx.ds, ctx.frame, g_color, g_D)
        return (None, None, None, g["cell_pos"], None, None, g["cell_v_sh"], g["means"], g["scales"], g["rots"],
                g["opacities"], g["sh"])


class L1SsimLoss(torch.autograd.Function):
    """The training loss (1 - lam) l1 + lam (1 - SSIM) of a rendered image
    against a fixed target, by the library: the forward computes the loss and
    dL/dimage in one call, the backward scales that gradient by the incoming
    one.  Inputs: renderer, image [C, H, W], target [C, H, W] (no gradient),
    lam.  Returns a 0-dim tensor."""

    @staticmethod
    def forward(ctx, renderer, image, target, lam=0.2):
        loss, g = renderer.loss_l1_ssim(image.detach(), target.detach(), lam, grad=image.requires_grad)
        ctx.g = g
        return loss

    @staticmethod
    def backward(ctx, g_loss):
        g = ctx.g  # kept with the graph: a retained graph may be walked again
        return None, (g * g_loss if g is not None else None), None, None
