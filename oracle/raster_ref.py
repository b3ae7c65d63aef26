"""Reference differentiable rasteriser -- TEST INFRASTRUCTURE ONLY.

Plain PyTorch, CPU, FP64, dense over (pixel, Gaussian) per view, so autograd
gives the reference gradient of the refinement's renderer (Sec. 4.6 trains
the relocated Gaussians with the 3DGS objective; Sec. 3.1 gives the
projection and depth-ordered blending):

  Sigma_3D = R S S^T R^T, Sigma_2D = J W Sigma_3D W^T J^T (Eq. 1),
  alpha = min(0.99, o exp(power)), skipped below 1/255, blending front to
  back with T, stopping before the Gaussian that would take T below 1e-4,
  colour = max(0, SH(view direction) . coefficients + 1/2),
  C = sum_i c_i alpha_i T_i + T_final bg.

Discrete decisions (which Gaussians a pixel's tile lists, their depth order,
the alpha threshold and termination) are constants of the forward pass, as in
any rasteriser; the tile rectangles and depth keys come from the oracle's
FP32 geometry decisions.
"""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
import synth


def sh_basis(deg, d):
    """Real SH basis (Condon-Shortley phase) up to degree 3 at unit
    directions d [...,3]; closed-form normalisation constants."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if deg > 0:
        c1 = math.sqrt(3.0 / (4.0 * pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if deg > 1:
        c2 = 0.5 * math.sqrt(15.0 / pi)
        c20 = 0.25 * math.sqrt(5.0 / pi)
        c22 = 0.25 * math.sqrt(15.0 / pi)
        out += [c2 * x * y, -c2 * y * z, c20 * (2 * z * z - x * x - y * y), -c2 * x * z, c22 * (x * x - y * y)]
    if deg > 2:
        c33 = 0.25 * math.sqrt(35.0 / (2.0 * pi))
        c32 = 0.5 * math.sqrt(105.0 / pi)
        c31 = 0.25 * math.sqrt(21.0 / (2.0 * pi))
        c30 = 0.25 * math.sqrt(7.0 / pi)
        c32b = 0.25 * math.sqrt(105.0 / pi)
        out += [-c33 * y * (3 * x * x - y * y), c32 * x * y * z, -c31 * y * (4 * z * z - x * x - y * y),
                c30 * z * (2 * z * z - 3 * x * x - 3 * y * y), -c31 * x * (4 * z * z - x * x - y * y),
                c32b * z * (x * x - y * y), -c33 * x * (x * x - 3 * y * y)]
    return torch.stack(out, -1)


def quat_to_rot_t(q):
    q = q / q.norm(dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _order(geom, v):
    """Depth order of the view's valid Gaussians: ascending FP32 depth key,
    ties by index (a stable sort of the keys)."""
    idx = np.nonzero(geom.valid[v])[0]
    return idx[np.lexsort((idx, geom.key[v, idx]))]


def _geom_of(means, quats, log_scales, cams):
    n = means.shape[0]
    sc = synth.Scene(means=means.detach().numpy().astype(np.float32),
                     quats=quats.detach().numpy().astype(np.float32),
                     scales=np.exp(log_scales.detach().numpy().astype(np.float32)),
                     opacity=np.zeros(n, np.float32), rgb=np.zeros((n, 3), np.float32))
    return oracle.geometry(sc, cams)


def _project(means, S3, sh, deg, cam, dil, jclamp, sel):
    """Centre, conic and view colour of the Gaussians `sel` in one view
    (Eq. 1 with the low-pass dilation added before the inverse)."""
    dt = torch.float64
    R = torch.tensor(cam.R, dtype=dt)
    t = torch.tensor(cam.t, dtype=dt)
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    m = means[sel]
    p = m @ R.T + t
    pz = p[:, 2]
    limx, limy = jclamp * 0.5 * cam.W / fx, jclamp * 0.5 * cam.H / fy
    tx = torch.clamp(p[:, 0] / pz, -limx, limx)
    ty = torch.clamp(p[:, 1] / pz, -limy, limy)
    zero = torch.zeros_like(pz)
    J = torch.stack([torch.stack([fx / pz, zero, -fx * tx / pz], -1),
                     torch.stack([zero, fy / pz, -fy * ty / pz], -1)], -2)
    T = J @ R
    S2 = T @ S3[sel] @ T.transpose(-1, -2) + dil * torch.eye(2, dtype=dt)
    Q = torch.linalg.inv(S2)
    mu = torch.stack([fx * p[:, 0] / pz + cx, fy * p[:, 1] / pz + cy], -1)
    centre = -R.T @ t
    dirs = m - centre
    dirs = dirs / dirs.norm(dim=-1, keepdim=True)
    col = torch.clamp((sh_basis(deg, dirs)[..., None] * sh[sel]).sum(1) + 0.5, min=0.0)
    return mu, Q, col


def _composite(pix, mu, Q, o, col, rect, bg, alpha_min, alpha_max, t_min, margin_rel):
    """Front-to-back compositing of depth-ordered Gaussians at pixels
    pix [P,2]; returns colours [P,3], per pixel whether a discrete decision
    (alpha threshold, alpha clamp, termination) lies within margin_rel
    (relative) of flipping, and a bound on how far such flips can move the
    pixel's colour (slack [P]): including or dropping Gaussian i changes
    its own term alpha_i T_i c_i and scales everything behind it (at most
    T_i times the largest colour) by (1 - alpha_i), so each near-threshold
    decision moves any channel by at most 2 alpha_i T_i cmax; a clamp
    decision by at most 2 margin_rel T_i cmax; the terminating Gaussian
    (T_i alpha_i and the rest are below T_i) by at most 2 T_i cmax."""
    dt = torch.float64
    ptx = (pix[:, 0] // 16).long()[:, None]
    pty = (pix[:, 1] // 16).long()[:, None]
    inrect = (ptx >= rect[None, :, 0]) & (ptx < rect[None, :, 2]) & (pty >= rect[None, :, 1]) & \
             (pty < rect[None, :, 3])
    d = pix[:, None, :] - mu[None, :, :]                                   # [P,K,2]
    power = -0.5 * (Q[None, :, 0, 0] * d[..., 0] ** 2 + Q[None, :, 1, 1] * d[..., 1] ** 2) - \
        Q[None, :, 0, 1] * d[..., 0] * d[..., 1]
    raw = o[None, :] * torch.exp(power)
    al = torch.clamp(raw, max=alpha_max)
    use = inrect & (power <= 0) & (al >= alpha_min)
    al = torch.where(use, al, torch.zeros_like(al))
    # termination: first Gaussian whose inclusion takes T below t_min
    with torch.no_grad():
        Tin = torch.cumprod(1.0 - al, dim=1)
        stop = use & (Tin < t_min)
        K = stop.shape[1]
        first = torch.full((stop.shape[0],), K)
        if K > 0:
            first = torch.where(stop.any(1), stop.float().argmax(1), first)
        ar = torch.arange(K)[None, :]
        keep = ar < first[:, None]
        upto = ar <= first[:, None]
        rawd = raw.detach()
        marg = inrect & upto & (power.detach() <= 0) & (
            ((rawd / alpha_min - 1).abs() < margin_rel) | ((rawd / alpha_max - 1).abs() < margin_rel) |
            (use & ((Tin / t_min - 1).abs() < margin_rel)))
        marginal = marg.any(1)
        Tfront = torch.cat([torch.ones_like(al[:, :1]), Tin[:, :-1]], 1)
        cmax = float(col.detach().abs().max()) if col.numel() else 0.0
        cmax = max(cmax, max(abs(float(x)) for x in bg))
        live = inrect & upto & (power.detach() <= 0)
        a_m = live & ((rawd / alpha_min - 1).abs() < margin_rel)
        c_m = live & ((rawd / alpha_max - 1).abs() < margin_rel)
        t_m = use & upto & ((Tin / t_min - 1).abs() < margin_rel)
        slack = 2.0 * cmax * (Tfront * (a_m * rawd.clamp(max=alpha_max) * (1 + margin_rel) +
                                        c_m * margin_rel + t_m)).sum(1)
    al = torch.where(keep, al, torch.zeros_like(al))
    Tex = torch.cat([torch.ones_like(al[:, :1]), torch.cumprod(1.0 - al, dim=1)[:, :-1]], 1)
    w = al * Tex
    Tfin = torch.prod(1.0 - al, dim=1)
    C = w @ col + Tfin[:, None] * torch.tensor(bg, dtype=dt)[None, :]
    return C, marginal, slack


def render(means, quats, log_scales, logit_opacity, sh, cams, bg=(0.0, 0.0, 0.0), geom=None, pixels=None,
           dil=0.3, jclamp=1.3, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, margin_rel=1e-3,
           return_marginal=False, return_slack=False):
    """FP64 reference colours (torch, differentiable).

    Dense images [V,H,W,3] when pixels is None; else pixels = (v, x, y)
    integer arrays and the result is [P,3] in that order.  geom: oracle
    Geometry holding the FP32 decisions (tile rectangles, depth keys);
    computed from the inputs (scales = exp(log_scales) in FP32) when None.
    With return_marginal, also a boolean mask (same leading shape) of
    pixels holding a decision within margin_rel of flipping; with
    return_slack as well, the bound on the colour change such flips can
    cause (see _composite)."""
    dt = torch.float64
    if geom is None:
        geom = _geom_of(means, quats, log_scales, cams)
    s = torch.exp(log_scales)
    o = torch.sigmoid(logit_opacity)
    Rq = quat_to_rot_t(quats)
    M = Rq * s[:, None, :]
    S3 = M @ M.transpose(-1, -2)
    deg = int(round(math.sqrt(sh.shape[1]))) - 1
    args = (bg, alpha_min, alpha_max, t_min, margin_rel)
    if pixels is None:
        imgs, margs, slacks = [], [], []
        for v, cam in enumerate(cams):
            order = torch.tensor(_order(geom, v).astype(np.int64))
            mu, Q, col = _project(means, S3, sh, deg, cam, dil, jclamp, order)
            rect = torch.tensor(geom.rect[v][order.numpy()].astype(np.int64))
            H, W = cam.H, cam.W
            yy, xx = torch.meshgrid(torch.arange(H, dtype=dt), torch.arange(W, dtype=dt), indexing="ij")
            pix = torch.stack([xx.reshape(-1), yy.reshape(-1)], -1)
            C, mg, sl = _composite(pix, mu, Q, o[order], col, rect, *args)
            imgs.append(C.reshape(H, W, 3))
            margs.append(mg.reshape(H, W))
            slacks.append(sl.reshape(H, W))
        out, marg, slack = torch.stack(imgs, 0), torch.stack(margs, 0), torch.stack(slacks, 0)
    else:
        pv, px, py = (np.asarray(a, np.int64) for a in pixels)
        out = [None] * len(pv)
        marg = torch.zeros(len(pv), dtype=torch.bool)
        slack = torch.zeros(len(pv), dtype=dt)
        for v in np.unique(pv):
            at = np.nonzero(pv == v)[0]
            order = _order(geom, v)
            rect_all = geom.rect[v][order].astype(np.int64)
            tx, ty = px[at] // 16, py[at] // 16
            cand = np.zeros(len(order), bool)
            for a_, b_ in set(zip(tx.tolist(), ty.tolist())):
                cand |= (rect_all[:, 0] <= a_) & (a_ < rect_all[:, 2]) & (rect_all[:, 1] <= b_) & (b_ < rect_all[:, 3])
            sel = torch.tensor(order[cand])
            mu, Q, col = _project(means, S3, sh, deg, cams[v], dil, jclamp, sel)
            pix = torch.tensor(np.stack([px[at], py[at]], -1).astype(np.float64))
            C, mg, sl = _composite(pix, mu, Q, o[sel], col, torch.tensor(rect_all[cand]), *args)
            for j, i in enumerate(at):
                out[i] = C[j]
            marg[torch.tensor(at)] = mg
            slack[torch.tensor(at)] = sl
        out = torch.stack(out, 0)
    if return_slack:
        return out, marg, slack
    return (out, marg) if return_marginal else out


# ---------------------------------------------------------------------------
# 3DGS objective (Sec. 4.6: the refinement uses the original 3DGS training):
# L = (1 - lambda) L1 + lambda (1 - SSIM), SSIM with an 11x11 Gaussian window
# (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, zero padding, mean over pixels and
# channels of every image.
# ---------------------------------------------------------------------------
SSIM_WIN, SSIM_SIGMA, SSIM_C1, SSIM_C2, DSSIM_LAMBDA = 11, 1.5, 0.01 ** 2, 0.03 ** 2, 0.2


def gaussian_window(n=SSIM_WIN, sigma=SSIM_SIGMA):
    x = torch.arange(n, dtype=torch.float64) - (n - 1) / 2
    g = torch.exp(-x * x / (2 * sigma * sigma))
    return g / g.sum()


def ssim(img, tgt):
    """Mean SSIM of images [..., H, W, C] (torch, differentiable, FP64)."""
    return ssim_map(img, tgt).mean()


def ssim_map(img, tgt):
    """Per-pixel SSIM [B*C, 1, H, W] of images [..., H, W, C]."""
    g = gaussian_window()
    w2 = (g[:, None] * g[None, :])[None, None]                    # [1,1,11,11]
    x = img.reshape(-1, *img.shape[-3:]).permute(0, 3, 1, 2).reshape(-1, 1, *img.shape[-3:-1])
    y = tgt.reshape(-1, *tgt.shape[-3:]).permute(0, 3, 1, 2).reshape(-1, 1, *tgt.shape[-3:-1])
    conv = lambda a: torch.nn.functional.conv2d(a, w2, padding=SSIM_WIN // 2)
    mx, my = conv(x), conv(y)
    sxx = conv(x * x) - mx * mx
    syy = conv(y * y) - my * my
    sxy = conv(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def loss_3dgs(img, tgt, lam=DSSIM_LAMBDA):
    return (1 - lam) * (img - tgt).abs().mean() + lam * (1 - ssim(img, tgt))
