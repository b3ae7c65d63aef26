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


def render(means, quats, log_scales, logit_opacity, sh, cams, bg=(0.0, 0.0, 0.0), geom=None,
           near=0.2, dil=0.3, jclamp=1.3, alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4):
    """FP64 reference images [V,H,W,3] (torch, differentiable).

    geom: oracle.Geometry for the FP32 decisions; computed from the inputs
    (scales = exp(log_scales) in FP32) when None."""
    dt = torch.float64
    N = means.shape[0]
    if geom is None:
        sc = synth.Scene(means=means.detach().numpy().astype(np.float32),
                         quats=quats.detach().numpy().astype(np.float32),
                         scales=np.exp(log_scales.detach().numpy().astype(np.float32)),
                         opacity=np.zeros(N, np.float32), rgb=np.zeros((N, 3), np.float32))
        geom = oracle.geometry(sc, cams)
    s = torch.exp(log_scales)
    o = torch.sigmoid(logit_opacity)
    Rq = quat_to_rot_t(quats)
    M = Rq * s[:, None, :]
    S3 = M @ M.transpose(-1, -2)
    k = sh.shape[1]
    deg = int(round(math.sqrt(k))) - 1
    imgs = []
    for v, cam in enumerate(cams):
        R = torch.tensor(cam.R, dtype=dt)
        t = torch.tensor(cam.t, dtype=dt)
        fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
        cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
        p = means @ R.T + t
        pz = p[:, 2]
        limx, limy = jclamp * 0.5 * cam.W / fx, jclamp * 0.5 * cam.H / fy
        tx = torch.clamp(p[:, 0] / pz, -limx, limx)
        ty = torch.clamp(p[:, 1] / pz, -limy, limy)
        zero = torch.zeros_like(pz)
        J = torch.stack([torch.stack([fx / pz, zero, -fx * tx / pz], -1),
                         torch.stack([zero, fy / pz, -fy * ty / pz], -1)], -2)
        T = J @ R
        S2 = T @ S3 @ T.transpose(-1, -2) + dil * torch.eye(2, dtype=dt)
        Q = torch.linalg.inv(S2)
        mu = torch.stack([fx * p[:, 0] / pz + cx, fy * p[:, 1] / pz + cy], -1)
        centre = -R.T @ t
        dirs = means - centre
        dirs = dirs / dirs.norm(dim=-1, keepdim=True)
        col = torch.clamp(torch.einsum("nk,nkc->nc", sh_basis(deg, dirs), sh) + 0.5, min=0.0)
        H, W = cam.H, cam.W
        yy, xx = torch.meshgrid(torch.arange(H, dtype=dt), torch.arange(W, dtype=dt), indexing="ij")
        pix = torch.stack([xx.reshape(-1), yy.reshape(-1)], -1)            # [P,2]
        valid = torch.tensor(geom.valid[v] != 0)
        idx = np.nonzero(geom.valid[v])[0]
        order = idx[np.lexsort((idx, geom.key[v, idx]))]
        order_t = torch.tensor(order.astype(np.int64))
        rect = torch.tensor(geom.rect[v][order].astype(np.int64))        # [K,4]
        ptx = (pix[:, 0] // 16).long()[:, None]
        pty = (pix[:, 1] // 16).long()[:, None]
        inrect = (ptx >= rect[None, :, 0]) & (ptx < rect[None, :, 2]) & (pty >= rect[None, :, 1]) & \
                 (pty < rect[None, :, 3])
        d = pix[:, None, :] - mu[order_t][None, :, :]                       # [P,K,2]
        Qo = Q[order_t]
        power = -0.5 * (Qo[None, :, 0, 0] * d[..., 0] ** 2 + Qo[None, :, 1, 1] * d[..., 1] ** 2) - \
            Qo[None, :, 0, 1] * d[..., 0] * d[..., 1]
        al = torch.clamp(o[order_t][None, :] * torch.exp(power), max=alpha_max)
        use = inrect & (power <= 0) & (al >= alpha_min)
        al = torch.where(use, al, torch.zeros_like(al))
        # termination: first Gaussian whose inclusion takes T below t_min
        with torch.no_grad():
            Tin = torch.cumprod(1.0 - al, dim=1)
            stop = use & (Tin < t_min)
            first = torch.where(stop.any(1), stop.float().argmax(1), torch.full((stop.shape[0],), stop.shape[1]))
            keep = torch.arange(al.shape[1])[None, :] < first[:, None]
        al = torch.where(keep, al, torch.zeros_like(al))
        Tex = torch.cat([torch.ones_like(al[:, :1]), torch.cumprod(1.0 - al, dim=1)[:, :-1]], 1)
        w = al * Tex
        Tfin = torch.prod(1.0 - al, dim=1)
        C = w @ col[order_t] + Tfin[:, None] * torch.tensor(bg, dtype=dt)[None, :]
        imgs.append(C.reshape(H, W, 3))
        del valid
    return torch.stack(imgs, 0)
