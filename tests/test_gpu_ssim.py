"""GPU parity of the 3DGS objective (tg_l1_loss_grad + tg_ssim_loss_grad,
through `Loss3DGS`) and of the two-rate Adam (tg_adam_step_rows), against the
FP64 reference objective of oracle/raster_ref.py and its autograd gradient.

Tolerances: the SSIM variance E[x^2] - mu^2 cancels, which amplifies FP32
rounding by up to mu^2 / (sigma^2 + C2) (about 1e3 at mu = 0.5 on flat
regions); with ~250 FP32 operations per pixel this bounds the gradient error
by 1e-3 of the largest gradient plus 1e-3 relative, and the loss (a mean of
SSIM values near 1, weighted by 0.2) by 5e-5."""
import math

import numpy as np
import pytest
import torch

import synth
from helpers import log
from oracle import raster_ref

pytestmark = pytest.mark.gpu


def _images(kind, shape, seed):
    rng = np.random.default_rng(seed)
    if kind == "noise":
        return rng.random(shape), rng.random(shape)
    if kind == "smooth":
        # flat regions (sigma^2 well below C2), identical blocks (S = 1) and a step
        tgt = np.full(shape, 0.5)
        tgt[..., shape[-3] // 2:, :, :] = 0.25
        img = tgt + 0.01 * rng.random(shape)
        img[..., : shape[-3] // 4, :, :] = tgt[..., : shape[-3] // 4, :, :]
        return img, tgt
    if kind == "saturated":
        # zeros and ones, as clamped renders produce
        return (rng.random(shape) < 0.5).astype(np.float64), (rng.random(shape) < 0.3).astype(np.float64)
    raise ValueError(kind)


def _ref(img, tgt):
    x = torch.tensor(img, dtype=torch.float64, requires_grad=True)
    loss = raster_ref.loss_3dgs(x, torch.tensor(tgt, dtype=torch.float64))
    loss.backward()
    return float(loss.detach()), x.grad.numpy()


def _gpu(img, tgt):
    from paper_2604_02586_amd.raster import Loss3DGS
    x = torch.tensor(img, dtype=torch.float32, device="cuda", requires_grad=True)
    loss = Loss3DGS.apply(x, torch.tensor(tgt, dtype=torch.float32, device="cuda"))
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), x.grad.cpu().double().numpy()


def _compare(got, ref, tag):
    (lg, gg), (lr, gr) = got, ref
    d = np.abs(gg - gr)
    scale = np.abs(gr).max()
    log(f"[{tag}] loss {lg:.7f} vs {lr:.7f}; max |dgrad| {d.max():.3e} (max |grad| {scale:.3e})")
    assert abs(lg - lr) <= 5e-5
    assert (d <= 1e-3 * scale + 1e-3 * np.abs(gr)).all()


CASES = {
    # ragged 16x16 tiles, several images
    "noise_ragged": ("noise", (3, 70, 53, 3), 1),
    "smooth": ("smooth", (2, 64, 48, 3), 2),
    "saturated": ("saturated", (1, 33, 47, 3), 3),
    # smaller than the 11x11 window in both directions
    "tiny": ("noise", (2, 5, 7, 3), 4),
    # one image, several tiles, no batch dimension
    "single": ("noise", (40, 36, 3), 5),
}


@pytest.mark.parametrize("case", list(CASES))
def test_loss_3dgs_matches_reference(case):
    kind, shape, seed = CASES[case]
    img, tgt = _images(kind, shape, seed)
    _compare(_gpu(img, tgt), _ref(img, tgt), case)


def test_identical_images():
    """SSIM of an image with itself is 1 and the gradient of both terms is 0."""
    img, _ = _images("noise", (2, 40, 40, 3), 6)
    lg, gg = _gpu(img, img)
    assert abs(lg) <= 1e-6
    # a non-trivial pair's gradient is O(1 / n) per element (about 2.5 / n
    # for uniform noise); the exact zero cancels to FP32 rounding
    assert np.abs(gg).max() <= 1e-4 / img.size


def test_full_size_sampled_views():
    """16 views of 1352x1014 (the refinement workload's image stack) in one
    call; two views against the reference (the objective is a sum over views,
    each normalised by the whole stack's element count)."""
    V, H, W = 16, 1014, 1352
    rng = np.random.default_rng(7)
    # rendered-like content: smooth gradients plus noise, clamped to [0, 1]
    yy, xx = np.mgrid[0:H, 0:W] / max(H, W)
    base = np.stack([np.sin(3 * xx + v) * np.cos(2 * yy) for v in range(V)])[..., None] * 0.4 + 0.5
    img = np.clip(base + 0.05 * rng.standard_normal((V, H, W, 3)), 0, 1).astype(np.float32)
    tgt = np.clip(base + 0.05 * rng.standard_normal((V, H, W, 3)), 0, 1).astype(np.float32)
    log(f"full size V={V} {W}x{H}")
    lg, gg = _gpu(img, tgt)
    n = img.size
    lam = raster_ref.DSSIM_LAMBDA
    for v in (0, V - 1):
        x = torch.tensor(img[v], dtype=torch.float64, requires_grad=True)
        y = torch.tensor(tgt[v], dtype=torch.float64)
        part = (1 - lam) * (x - y).abs().sum() / n - lam * raster_ref.ssim_map(x, y).sum() / n
        part.backward()
        d = np.abs(gg[v] - x.grad.numpy())
        scale = np.abs(x.grad.numpy()).max()
        log(f"view {v}: max |dgrad| {d.max():.3e} (max |grad| {scale:.3e})")
        assert (d <= 1e-3 * scale + 1e-3 * np.abs(x.grad.numpy())).all()
    assert math.isfinite(lg) and 0.0 < lg < 1.0


def test_adam_rows_matches_formula():
    """Two learning rates by position in a row (3DGS: DC colour vs higher SH
    bands), three steps of bias-corrected Adam (Kingma & Ba, Alg. 1)."""
    from paper_2604_02586_amd.raster import Adam
    rng = np.random.default_rng(8)
    N, K = 1001, 16
    p0 = rng.standard_normal((N, K, 3)).astype(np.float32)
    gs = [rng.standard_normal((N, K, 3)).astype(np.float32) for _ in range(3)]
    pt = torch.tensor(p0, device="cuda")
    opt = Adam([pt], lr=[(2.5e-3, 2.5e-3 / 20, 3 * K, 3)], eps=1e-15)
    lr = np.full((N, K, 3), 2.5e-3 / 20)
    lr[:, 0, :] = 2.5e-3
    pr, m, v = p0.astype(np.float64), np.zeros_like(lr), np.zeros_like(lr)
    for t, g in enumerate(gs, 1):
        pt.grad = torch.tensor(g, device="cuda")
        opt.step()
        m = 0.9 * m + 0.1 * g
        v = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
        pr = pr - lr * (m / (1 - 0.9 ** t)) / (np.sqrt(v / (1 - 0.999 ** t)) + 1e-15)
    np.testing.assert_allclose(pt.cpu().numpy(), pr, rtol=0, atol=5e-6)


def test_refinement_3dgs_recipe_reduces_loss():
    """The 3DGS recipe (objective and per-parameter rates) from a perturbed
    copy lowers the 3DGS objective against reference-rendered targets."""
    from paper_2604_02586_amd.raster import RasterContext, refine
    wl = synth.make_refine_workload("refine_fd", n=800, views=4, width=96, height=96, seed=31)
    rp = [torch.tensor(np.asarray(wl.gt[k], np.float64))
          for k in ("means", "quats", "log_scales", "logit_opacity", "sh")]
    target = raster_ref.render(*rp, wl.cams).float().cuda()
    gp = [torch.tensor(np.asarray(wl.init[k], np.float32), device="cuda", requires_grad=True)
          for k in ("means", "quats", "log_scales", "logit_opacity", "sh")]
    rc = RasterContext(wl.cams, wl.meta["n"])
    losses = refine(gp, rc, target, iters=150, log_every=1, recipe="3dgs")
    log(f"3dgs loss {losses[0]:.5f} -> {losses[-1]:.5f}")
    assert all(math.isfinite(x) for x in losses)
    assert losses[-1] < 0.8 * losses[0]
