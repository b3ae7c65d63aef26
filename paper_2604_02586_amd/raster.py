"""Differentiable rasteriser and refinement loop over libtg (Sec. 4.6).

`Rasterize` is a torch.autograd.Function whose forward runs tg_preprocess
(SH colours, log-scales, logit opacities) -> tg_bin_sort -> tg_raster_fwd and
whose backward runs tg_raster_bwd -> tg_project_bwd; `L1Loss` wraps
tg_l1_loss_grad; `Loss3DGS` (the 3DGS objective (1 - lambda) L1 +
lambda (1 - SSIM)) wraps tg_l1_loss_grad + tg_ssim_loss_grad; `Adam` wraps
tg_adam_step / tg_adam_step_rows.  `refine` runs either L1 + one learning rate
or the 3DGS recipe (objective, per-parameter learning rates, exponentially
decayed position rate).  Torch holds the memory and the autograd graph; every
arithmetic step runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .api import BinTensors, GaussianTensors, SplatTensors, _ptr, bin_sort, bin_sort_ws_bytes, preprocess, stream_ptr
from ._lib import check, lib

__all__ = ["RasterContext", "Rasterize", "L1Loss", "Loss3DGS", "Adam", "rasterize", "refine", "lr_3dgs",
           "scene_extent"]

DSSIM_LAMBDA = 0.2


class RasterContext:
    """Buffers for rendering N Gaussians into V views of one resolution."""

    def __init__(self, cams, n, device="cuda", bg=(0.0, 0.0, 0.0), params=None, capacity=None):
        self.cams = cams if isinstance(cams, ctypes.Array) else _lib.cameras(cams)
        self.V = len(self.cams)
        self.N = int(n)
        self.W, self.H = int(self.cams[0].width), int(self.cams[0].height)
        self.device = torch.device(device)
        self.params = params if params is not None else _lib.default_params()
        self.bg = (ctypes.c_float * 3)(*bg)
        L = lib()
        self.n_cells = int(L.tg_num_cells(self.cams, self.V, self.N, ctypes.byref(self.params)))
        self.splats = SplatTensors.alloc(self.V, self.N, self.device, colors=True)
        self._alloc_bins(capacity or max(1024, 4 * self.N * self.V))
        shp = (self.V, self.H, self.W)
        self.image = torch.empty(*shp, 3, dtype=torch.float32, device=self.device)
        self.n_proc = torch.empty(*shp, dtype=torch.int32, device=self.device)
        self.grad2d = torch.empty(self.V, self.N, 9, dtype=torch.float32, device=self.device)
        # forward count: a backward must follow its own forward (the buffers
        # above are reused by every forward through this context)
        self.gen = 0
        # pair-count check without a host sync per iteration: each binning
        # copies its count and overflow flag to pinned memory behind an
        # event; the next forward reads the previous one (already finished)
        self._check = torch.zeros(2, dtype=torch.int64).pin_memory()
        self._check_ev = None
        self._sized = False
        # optional device int64 [5]: the forward adds (pairs evaluated, pairs
        # contributing), the backward (pixel steps, pairs evaluated, pairs
        # contributing) -- see count_pairs
        self.pair_counts = None

    def count_pairs(self, on=True):
        """Switch the pair counters of the rasteriser on (zeroed) or off."""
        self.pair_counts = torch.zeros(5, dtype=torch.int64, device=self.device) if on else None

    def _alloc_bins(self, capacity):
        self.bins = BinTensors.alloc(self.V, self.N, self.n_cells, capacity, self.device)
        self.ws = torch.empty(bin_sort_ws_bytes(self.N, self.cams, self.params, capacity), dtype=torch.uint8,
                              device=self.device)

    def _lagged_check(self):
        """Reads the previous binning's pair count (its event has long
        completed by the next iteration); raises if it overflowed, after
        growing the capacity for the next forward."""
        if self._check_ev is None:
            return
        self._check_ev.synchronize()
        self._check_ev = None
        if int(self._check[1]):
            need = int(self._check[0])
            self._alloc_bins(int(need * 1.25) + 1024)
            raise RuntimeError(f"pair-list overflow in the previous forward ({need} pairs, capacity too small): "
                               "its image and gradient were incomplete; the capacity has been raised")

    def forward(self, g: GaussianTensors, check_overflow=True):
        """Renders into self.image (valid until the next forward through this
        context).  The first forward sizes the pair list with a host sync;
        later ones check the previous forward's count without one."""
        if check_overflow:
            self._lagged_check()
        preprocess(g, self.cams, self.params, self.splats)
        bin_sort(self.splats, self.N, self.cams, self.params, self.bins, self.ws)
        if check_overflow and not self._sized:
            torch.cuda.current_stream().synchronize()
            need = int(self.bins.n_pairs.item())
            if int(self.bins.overflow.item()) or need * 1.25 > self.bins.capacity:
                self._alloc_bins(int(need * 1.25) + 1024)
                bin_sort(self.splats, self.N, self.cams, self.params, self.bins, self.ws)
            self._sized = True
        elif check_overflow:
            self._check[0].copy_(self.bins.n_pairs[0], non_blocking=True)
            self._check[1].copy_(self.bins.overflow[0].to(torch.int64), non_blocking=True)
            self._check_ev = torch.cuda.Event()
            self._check_ev.record(torch.cuda.current_stream())
        self.gen += 1
        sc, bc = self.splats.c(), self.bins.c()
        if self.pair_counts is not None:
            check("tg_raster_fwd_counted", lib().tg_raster_fwd_counted(
                ctypes.byref(sc), ctypes.byref(bc), self.N, self.cams, self.V, self.bg, ctypes.byref(self.params),
                _ptr(self.image), None, _ptr(self.n_proc), _ptr(self.pair_counts), stream_ptr()))
        else:
            check("tg_raster_fwd", lib().tg_raster_fwd(ctypes.byref(sc), ctypes.byref(bc), self.N, self.cams, self.V,
                                                       self.bg, ctypes.byref(self.params), _ptr(self.image), None,
                                                       _ptr(self.n_proc), stream_ptr()))
        return self.image

    def backward(self, g: GaussianTensors, dimage: torch.Tensor, grads: GaussianTensors):
        self.grad2d.zero_()
        sc, bc = self.splats.c(), self.bins.c()
        dimage = dimage.contiguous()
        if self.pair_counts is not None:
            check("tg_raster_bwd_counted", lib().tg_raster_bwd_counted(
                ctypes.byref(sc), ctypes.byref(bc), self.N, self.cams, self.V, _ptr(self.image), _ptr(dimage),
                _ptr(self.n_proc), ctypes.byref(self.params), _ptr(self.grad2d), _ptr(self.pair_counts[2:]),
                stream_ptr()))
        else:
            check("tg_raster_bwd", lib().tg_raster_bwd(ctypes.byref(sc), ctypes.byref(bc), self.N, self.cams, self.V,
                                                       _ptr(self.image), _ptr(dimage), _ptr(self.n_proc),
                                                       ctypes.byref(self.params), _ptr(self.grad2d), stream_ptr()))
        gc, grc = g.c(), grads.c()
        check("tg_project_bwd", lib().tg_project_bwd(ctypes.byref(gc), ctypes.byref(sc), self.N, self.cams, self.V,
                                                     _ptr(self.grad2d), ctypes.byref(self.params), ctypes.byref(grc),
                                                     stream_ptr()))


class Rasterize(torch.autograd.Function):
    """image[V,H,W,3] = render(means, quats, log_scales, logit_opacity, sh)."""

    @staticmethod
    def forward(ctx, means, quats, log_scales, logit_opacity, sh, rc: RasterContext):
        deg = int(round((sh.shape[1]) ** 0.5)) - 1
        g = GaussianTensors(means.contiguous(), quats.contiguous(), log_scales.contiguous(),
                            logit_opacity.contiguous(), sh.contiguous(), deg, 1, 1)
        img = rc.forward(g)
        ctx.rc, ctx.g, ctx.gen = rc, g, rc.gen
        # an alias of the context's image buffer (no copy), valid until the
        # context's next forward
        return img.detach()

    @staticmethod
    def backward(ctx, dimage):
        if ctx.gen != ctx.rc.gen:
            raise RuntimeError("this RasterContext ran another forward before this backward; its buffers hold the "
                               "later render (use one RasterContext per render that is back-propagated)")
        g = ctx.g
        grads = GaussianTensors(torch.empty_like(g.means), torch.empty_like(g.quats), torch.empty_like(g.scales),
                                torch.empty_like(g.opacity), torch.empty_like(g.sh), g.sh_degree, 1, 1)
        ctx.rc.backward(g, dimage, grads)
        return grads.means, grads.quats, grads.scales, grads.opacity, grads.sh, None


class L1Loss(torch.autograd.Function):
    """mean |image - target| with the gradient from tg_l1_loss_grad."""

    @staticmethod
    def forward(ctx, image, target):
        image, target = image.contiguous(), target.contiguous()
        n = image.numel()
        grad = torch.empty_like(image)
        loss = torch.zeros(1, dtype=torch.float32, device=image.device)
        check("tg_l1_loss_grad", lib().tg_l1_loss_grad(_ptr(image), _ptr(target), n, ctypes.c_float(1.0 / n),
                                                       _ptr(grad), _ptr(loss), stream_ptr()))
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        (grad,) = ctx.saved_tensors
        return _chain(grad, gl), None


def _chain(grad, gl):
    """grad * gl with gl a device scalar (tg_scale_by; no host read)."""
    out = torch.empty_like(grad)
    gl = gl.reshape(1).to(torch.float32).contiguous()
    check("tg_scale_by", lib().tg_scale_by(_ptr(out), _ptr(grad), grad.numel(), _ptr(gl), stream_ptr()))
    return out


class Loss3DGS(torch.autograd.Function):
    """(1 - lam) mean|image - target| + lam (1 - mean SSIM(image, target)) over
    images [..., H, W, 3]; the gradient comes from tg_l1_loss_grad followed by
    tg_ssim_loss_grad (which adds the SSIM term's share)."""

    @staticmethod
    def forward(ctx, image, target, lam=DSSIM_LAMBDA):
        image, target = image.contiguous(), target.contiguous()
        H, W = image.shape[-3], image.shape[-2]
        if image.shape[-1] != 3 or target.shape != image.shape:
            raise ValueError("images must be [..., H, W, 3] of one shape")
        n = image.numel()
        B = n // (H * W * 3) if n else 0
        grad = torch.empty_like(image)
        sums = torch.zeros(2, dtype=torch.float32, device=image.device)
        st = stream_ptr()
        check("tg_l1_loss_grad", lib().tg_l1_loss_grad(_ptr(image), _ptr(target), n, ctypes.c_float((1 - lam) / max(n, 1)),
                                                       _ptr(grad), _ptr(sums), st))
        wsb = ctypes.c_size_t(0)
        check("tg_ssim_loss_grad", lib().tg_ssim_loss_grad(None, None, B, H, W, ctypes.c_float(0), None, None, None,
                                                           ctypes.byref(wsb), st))
        ws = torch.empty(max(wsb.value, 1), dtype=torch.uint8, device=image.device)
        check("tg_ssim_loss_grad", lib().tg_ssim_loss_grad(_ptr(image), _ptr(target), B, H, W,
                                                           ctypes.c_float(-lam / max(n, 1)), _ptr(grad),
                                                           _ptr(sums[1:]), _ptr(ws), ctypes.byref(wsb), st))
        ctx.save_for_backward(grad)
        # sums = [(1 - lam) L1, sum of the SSIM map]; the objective is
        # sums[0] + lam - (lam / n) sums[1]
        loss = torch.empty(1, dtype=torch.float32, device=image.device)
        w = (ctypes.c_float * 2)(1.0, -lam / max(n, 1))
        check("tg_scalar_affine", lib().tg_scalar_affine(_ptr(loss), _ptr(sums), 2, w, ctypes.c_float(lam), st))
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        (grad,) = ctx.saved_tensors
        return _chain(grad, gl), None, None


def rasterize(means, quats, log_scales, logit_opacity, sh, rc):
    return Rasterize.apply(means, quats, log_scales, logit_opacity, sh, rc)


class Adam:
    """Adam over a list of tensors; the update runs in tg_adam_step.

    lr: one rate, or one entry per tensor, each a float or a tuple
    (lr_head, lr_tail, row, head) for tg_adam_step_rows (the first `head` of
    every `row` floats step with lr_head).  `lr` may be reassigned between
    steps (learning-rate schedules)."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-15):
        self.params = list(params)
        self.lr = list(lr) if isinstance(lr, (list, tuple)) else [lr] * len(self.params)
        if len(self.lr) != len(self.params):
            raise ValueError("one learning rate per tensor")
        self.b1, self.b2 = betas
        self.eps = eps
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def step(self):
        self.t += 1
        f = ctypes.c_float
        for p, m, v, lr in zip(self.params, self.m, self.v, self.lr):
            if p.grad is None:
                continue
            g = p.grad.contiguous()
            if isinstance(lr, tuple):
                lr_head, lr_tail, row, head = lr
                check("tg_adam_step_rows", lib().tg_adam_step_rows(
                    _ptr(p.data), _ptr(g), _ptr(m), _ptr(v), p.numel(), row, head, f(lr_head), f(lr_tail),
                    f(self.b1), f(self.b2), f(self.eps), self.t, stream_ptr()))
            else:
                check("tg_adam_step", lib().tg_adam_step(_ptr(p.data), _ptr(g), _ptr(m), _ptr(v), p.numel(), f(lr),
                                                         f(self.b1), f(self.b2), f(self.eps), self.t, stream_ptr()))

    def zero_grad(self):
        for p in self.params:
            p.grad = None


def scene_extent(cams):
    """3DGS's spatial learning-rate scale: 1.1 x the largest distance of a
    camera centre from the mean camera centre."""
    import numpy as np
    centres = np.stack([-np.asarray(c.R, np.float64).reshape(3, 3).T @ np.asarray(c.t, np.float64) for c in cams])
    d = np.linalg.norm(centres - centres.mean(0), axis=1).max()
    return 1.1 * float(d)


# 3DGS learning rates: position (scaled by the scene extent, decayed
# exponentially from init to final over max_steps), DC colour, higher SH bands
# (DC / 20), opacity, scale, rotation
LR_3DGS = dict(position_init=1.6e-4, position_final=1.6e-6, position_max_steps=30000, feature=2.5e-3,
               feature_rest_div=20.0, opacity=0.05, scaling=5e-3, rotation=1e-3)


def lr_3dgs(step, extent, sh_coeffs, cfg=LR_3DGS):
    """Per-tensor rates for (means, quats, log_scales, logit_opacity, sh) at
    optimiser step `step` (0-based)."""
    import math
    t = min(max(step / cfg["position_max_steps"], 0.0), 1.0)
    pos = math.exp((1 - t) * math.log(cfg["position_init"]) + t * math.log(cfg["position_final"])) * extent
    f = cfg["feature"]
    sh = (f, f / cfg["feature_rest_div"], 3 * sh_coeffs, 3)
    return [pos, cfg["rotation"], cfg["scaling"], cfg["opacity"], sh]


def refine(params, rc: RasterContext, targets, iters=100, lr=1e-3, log_every=0, recipe="l1", extent=None):
    """Refinement of (means, quats, log_scales, logit_opacity, sh) against
    targets [V,H,W,3].  recipe "l1": L1 + Adam at one rate `lr`; recipe
    "3dgs": the 3DGS objective and per-parameter rates (`lr` unused; extent
    defaults to scene_extent of the context's cameras)."""
    if recipe not in ("l1", "3dgs"):
        raise ValueError(f"unknown recipe {recipe!r}")
    if recipe == "3dgs":
        extent = scene_extent(rc.cams) if extent is None else extent
        K = params[4].shape[1]
        opt = Adam(params, lr=lr_3dgs(0, extent, K))
    else:
        opt = Adam(params, lr=lr)
    losses = []
    for it in range(iters):
        if recipe == "3dgs":
            opt.lr = lr_3dgs(it, extent, K)
        img = rasterize(*params, rc)
        loss = Loss3DGS.apply(img, targets) if recipe == "3dgs" else L1Loss.apply(img, targets)
        opt.zero_grad()
        loss.backward()
        opt.step()
        if log_every and (it % log_every == 0 or it == iters - 1):
            losses.append(float(loss.item()))
    return losses
