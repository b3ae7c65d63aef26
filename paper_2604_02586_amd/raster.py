"""Differentiable rasteriser and refinement loop over libtg (Sec. 4.6).

`Rasterize` is a torch.autograd.Function whose forward runs tg_preprocess
(SH colours, log-scales, logit opacities) -> tg_bin_sort -> tg_raster_fwd and
whose backward runs tg_raster_bwd -> tg_project_bwd; `L1Loss` wraps
tg_l1_loss_grad; `Adam` wraps tg_adam_step.  Torch holds the memory and the
autograd graph; every arithmetic step runs in the HIP kernels.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .api import BinTensors, GaussianTensors, SplatTensors, _ptr, bin_sort, bin_sort_ws_bytes, preprocess, stream_ptr
from ._lib import check, lib

__all__ = ["RasterContext", "Rasterize", "L1Loss", "Adam", "rasterize", "refine"]


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

    def _alloc_bins(self, capacity):
        self.bins = BinTensors.alloc(self.V, self.N, self.n_cells, capacity, self.device)
        self.ws = torch.empty(bin_sort_ws_bytes(self.N, self.cams, self.params, capacity), dtype=torch.uint8,
                              device=self.device)

    def forward(self, g: GaussianTensors, check_overflow=True):
        preprocess(g, self.cams, self.params, self.splats)
        bin_sort(self.splats, self.N, self.cams, self.params, self.bins, self.ws)
        if check_overflow:
            torch.cuda.current_stream().synchronize()
            if int(self.bins.overflow.item()):
                self._alloc_bins(int(int(self.bins.n_pairs.item()) * 1.1) + 1024)
                bin_sort(self.splats, self.N, self.cams, self.params, self.bins, self.ws)
        sc, bc = self.splats.c(), self.bins.c()
        check("tg_raster_fwd", lib().tg_raster_fwd(ctypes.byref(sc), ctypes.byref(bc), self.N, self.cams, self.V,
                                                   self.bg, ctypes.byref(self.params), _ptr(self.image), None,
                                                   _ptr(self.n_proc), stream_ptr()))
        return self.image

    def backward(self, g: GaussianTensors, dimage: torch.Tensor, grads: GaussianTensors):
        self.grad2d.zero_()
        sc, bc = self.splats.c(), self.bins.c()
        dimage = dimage.contiguous()
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
        img = rc.forward(g).clone()
        ctx.rc, ctx.g = rc, g
        return img

    @staticmethod
    def backward(ctx, dimage):
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
        return grad * gl, None


def rasterize(means, quats, log_scales, logit_opacity, sh, rc):
    return Rasterize.apply(means, quats, log_scales, logit_opacity, sh, rc)


class Adam:
    """Adam over a list of tensors; the update runs in tg_adam_step."""

    def __init__(self, params, lr=1e-3, betas=(0.9, 0.999), eps=1e-15):
        self.params = list(params)
        self.lr = lr if isinstance(lr, (list, tuple)) else [lr] * len(self.params)
        self.b1, self.b2 = betas
        self.eps = eps
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0

    def step(self):
        self.t += 1
        for p, m, v, lr in zip(self.params, self.m, self.v, self.lr):
            if p.grad is None:
                continue
            g = p.grad.contiguous()
            check("tg_adam_step", lib().tg_adam_step(_ptr(p.data), _ptr(g), _ptr(m), _ptr(v), p.numel(),
                                                     ctypes.c_float(lr), ctypes.c_float(self.b1),
                                                     ctypes.c_float(self.b2), ctypes.c_float(self.eps), self.t,
                                                     stream_ptr()))

    def zero_grad(self):
        for p in self.params:
            p.grad = None


def refine(params, rc: RasterContext, targets, iters=100, lr=1e-3, log_every=0):
    """L1 + Adam refinement of (means, quats, log_scales, logit_opacity, sh)."""
    opt = Adam(params, lr=lr)
    losses = []
    for it in range(iters):
        img = rasterize(*params, rc)
        loss = L1Loss.apply(img, targets)
        opt.zero_grad()
        loss.backward()
        opt.step()
        if log_every and (it % log_every == 0 or it == iters - 1):
            losses.append(float(loss.item()))
    return losses
