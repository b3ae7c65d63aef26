"""Seeded synthetic inputs for TrackerSplat motion transfer.

This module only *draws* inputs: Gaussian scenes, pinhole cameras, a
ground-truth 3D motion and per-pixel 2D track fields.  It holds none of the
method's arithmetic (no EWA covariance projection, no alpha compositing, no
least squares, no triangulation), so both the GPU path and the CPU oracle can
consume the same inputs without sharing any code that computes a result.

Workload shapes follow the paper's datasets (Sec. 5.1): view counts from 4 to
27, resolutions up to 1920x1080, dense per-pixel tracks of the first frame
(Sec. 3.2).  The datasets themselves are not available; these synthetic
scenes stand in for them.

Track fields here are *proxy-rendered*: for each pixel, the ray is
intersected with the scene's bounding sphere and the ground-truth motion field
is evaluated at that surface point and re-projected.  Noise, uniform outliers
and Bernoulli visibility are added as the workload asks.

Array conventions (all float32 unless noted):
  means [N,3]; quats [N,4] (w,x,y,z) with w >= 0; scales [N,3] (linear);
  opacity [N] in (0,1); rgb [N,3]; sh [N,48] (degree 3, channel-minor);
  camera: dict(R=[3,3] world->camera rows, t=[3], fx, fy, cx, cy, W, H),
  p_cam = R @ x + t, x right / y down / z forward;
  disp [V,H,W,2] = x' - x in pixels (pixel (row r, col c) sits at (c, r));
  vis [V,H,W] uint8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "Camera", "Motion", "Workload",
    "look_at_camera", "ring_cameras", "hemisphere_cameras",
    "random_gaussians", "per_gaussian_rigid_motion", "body_field_motion",
    "proxy_tracks", "make_workload", "camera_array", "WORKLOADS",
]


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class Camera:
    R: np.ndarray      # [3,3] float32, world -> camera
    t: np.ndarray      # [3] float32
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int

    @property
    def center(self) -> np.ndarray:
        R = self.R.astype(np.float64)
        return -R.T @ self.t.astype(np.float64)


@dataclass
class Scene:
    means: np.ndarray
    quats: np.ndarray
    scales: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray
    sh: np.ndarray | None = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])


@dataclass
class Motion:
    """Ground-truth per-Gaussian target state (for accuracy reports only)."""
    means: np.ndarray
    quats: np.ndarray
    scales: np.ndarray
    # optional field evaluator x[...,3] (float64) -> moved x (float64)
    field: object = None


@dataclass
class Workload:
    name: str
    scene: Scene
    cams: list
    motion: Motion
    disp: np.ndarray          # [V,H,W,2] float32
    vis: np.ndarray           # [V,H,W] uint8
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def look_at_camera(center, target, up, W, H, fov_x_deg) -> Camera:
    """Pinhole camera at `center` looking at `target`; OpenCV axes."""
    c = np.asarray(center, np.float64)
    f = np.asarray(target, np.float64) - c
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(r) < 1e-9:          # looking along `up`
        r = np.cross(f, np.array([1.0, 0.0, 0.0]))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0)
    t = -R @ c
    fx = 0.5 * W / math.tan(math.radians(fov_x_deg) * 0.5)
    return Camera(R=R.astype(np.float32), t=t.astype(np.float32),
                  fx=float(np.float32(fx)), fy=float(np.float32(fx)),
                  cx=float(np.float32((W - 1) * 0.5)), cy=float(np.float32((H - 1) * 0.5)),
                  W=int(W), H=int(H))


def ring_cameras(n, radius, W, H, fov_x_deg=60.0):
    """n cameras on the z = 0 circle, evenly spaced azimuths, up = +z."""
    cams = []
    for k in range(n):
        a = 2.0 * math.pi * k / n
        cams.append(look_at_camera([radius * math.cos(a), radius * math.sin(a), 0.0],
                                   [0, 0, 0], [0, 0, 1], W, H, fov_x_deg))
    return cams


def hemisphere_cameras(n, radius, W, H, fov_x_deg=60.0, elev_lo=10.0, elev_hi=80.0):
    """n cameras on the upper hemisphere (Fibonacci lattice in elevation band)."""
    cams = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    zlo, zhi = math.sin(math.radians(elev_lo)), math.sin(math.radians(elev_hi))
    for k in range(n):
        z = zlo + (zhi - zlo) * (k + 0.5) / n
        rr = math.sqrt(max(0.0, 1.0 - z * z))
        a = golden * k
        cams.append(look_at_camera([radius * rr * math.cos(a), radius * rr * math.sin(a), radius * z],
                                   [0, 0, 0], [0, 0, 1], W, H, fov_x_deg))
    return cams


def camera_array(cams) -> np.ndarray:
    """Pack cameras into the [V, 20] float32 layout of the C boundary.

    Layout per camera (80 bytes): R (9 float32, row-major), t (3 float32),
    fx, fy, cx, cy (float32), width, height (int32), two zero pads.
    """
    out = np.zeros((len(cams), 20), np.float32)
    iv = out.view(np.int32)
    for i, c in enumerate(cams):
        out[i, 0:9] = c.R.reshape(-1)
        out[i, 9:12] = c.t
        out[i, 12:16] = [c.fx, c.fy, c.cx, c.cy]
        iv[i, 16:18] = [c.W, c.H]
    return out


# --------------------------------------------------------------------------
# Gaussians
# --------------------------------------------------------------------------
def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q


def random_gaussians(rng, n, *, domain="cube", radius=1.0, log_s_lo=math.log(0.01),
                     log_s_hi=math.log(0.05), sh_degree=0) -> Scene:
    if domain == "cube":
        means = rng.uniform(-1.0, 1.0, (n, 3))
    elif domain == "ball":
        d = rng.standard_normal((n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = radius * rng.uniform(0.0, 1.0, n) ** (1.0 / 3.0)
        means = d * r[:, None]
    else:
        raise ValueError(domain)
    log_s = rng.uniform(log_s_lo, log_s_hi, (n, 3))
    quats = _unit_quats(rng, n)
    opacity = rng.uniform(0.1, 0.9, n)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    sh = None
    if sh_degree > 0:
        k = (sh_degree + 1) ** 2
        sh = (rng.standard_normal((n, k * 3)) * 0.2).astype(np.float32)
    return Scene(means=means.astype(np.float32), quats=quats.astype(np.float32),
                 scales=np.exp(log_s).astype(np.float32), opacity=opacity.astype(np.float32),
                 rgb=rgb.astype(np.float32), sh=sh)


# --------------------------------------------------------------------------
# ground-truth motion
# --------------------------------------------------------------------------
def _axis_angle_quat(axis, angle):
    axis = axis / np.linalg.norm(axis, axis=-1, keepdims=True)
    h = 0.5 * angle
    return np.concatenate([np.cos(h)[..., None], axis * np.sin(h)[..., None]], -1)


def _quat_mul(a, b):
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], -1)


def _quat_to_mat(q):
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(q, -1, 0)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def _pinhole(cam: Camera, X):
    """Pixel position of 3D points X[...,3] (float64) -- camera model only."""
    R = cam.R.astype(np.float64)
    p = X @ R.T + cam.t.astype(np.float64)
    z = p[..., 2]
    return np.stack([cam.fx * p[..., 0] / z + cam.cx, cam.fy * p[..., 1] / z + cam.cy], -1), z


def per_gaussian_rigid_motion(rng, scene: Scene, max_angle_deg=10.0, max_trans=0.1) -> Motion:
    """Each Gaussian rotates about its own centre and translates."""
    n = scene.n
    axis = rng.standard_normal((n, 3))
    ang = np.radians(rng.uniform(0.0, max_angle_deg, n))
    tdir = rng.standard_normal((n, 3))
    tdir /= np.linalg.norm(tdir, axis=1, keepdims=True)
    tmag = rng.uniform(0.0, max_trans, n)
    dq = _axis_angle_quat(axis, ang)
    q = _quat_mul(dq, scene.quats.astype(np.float64))
    q[q[:, 0] < 0] *= -1.0
    means = scene.means.astype(np.float64) + tdir * tmag[:, None]
    return Motion(means=means.astype(np.float32), quats=q.astype(np.float32),
                  scales=scene.scales.copy(), field=None)


class _BodyField:
    """Soft blend of K rigid bodies: x -> sum_k beta_k(x) (R_k (x - c_k) + c_k + t_k)."""

    def __init__(self, centers, quats, trans, sigma):
        self.c = centers
        self.q = quats
        self.t = trans
        self.R = _quat_to_mat(quats)
        self.sigma = sigma

    def weights(self, X):
        d2 = ((X[..., None, :] - self.c) ** 2).sum(-1)
        lw = -d2 / (2.0 * self.sigma ** 2)
        lw -= lw.max(-1, keepdims=True)
        w = np.exp(lw)
        return w / w.sum(-1, keepdims=True)

    def __call__(self, X):
        X = np.asarray(X, np.float64)
        b = self.weights(X)
        out = np.zeros_like(X)
        for k in range(self.c.shape[0]):
            out += b[..., k:k + 1] * ((X - self.c[k]) @ self.R[k].T + self.c[k] + self.t[k])
        return out

    def rotation(self, X):
        b = self.weights(np.asarray(X, np.float64))
        q = self.q.copy()
        q[np.einsum("kc,c->k", q, q[0]) < 0] *= -1.0       # sign-align to body 0
        qb = b @ q
        return qb / np.linalg.norm(qb, axis=-1, keepdims=True)


def body_field_motion(rng, scene: Scene, cams, *, n_bodies=8, ball_radius=2.0,
                      max_angle_deg=10.0, max_trans=0.2, cap_px=60.0, sigma=0.5) -> Motion:
    """Smooth motion field of soft-blended rigid bodies, scaled so that the
    largest projected mean displacement over all views is at most cap_px."""
    d = rng.standard_normal((n_bodies, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centers = d * (ball_radius * rng.uniform(0, 1, n_bodies) ** (1 / 3))[:, None]
    axes = rng.standard_normal((n_bodies, 3))
    angles = np.radians(rng.uniform(0, max_angle_deg, n_bodies))
    tdir = rng.standard_normal((n_bodies, 3))
    tdir /= np.linalg.norm(tdir, axis=1, keepdims=True)
    tmag = rng.uniform(0, max_trans, n_bodies)
    mu = scene.means.astype(np.float64)
    sub = mu if mu.shape[0] <= 20000 else mu[rng.choice(mu.shape[0], 20000, replace=False)]
    scale = 1.0
    for _ in range(4):
        f = _BodyField(centers, _axis_angle_quat(axes, angles * scale), tdir * (tmag * scale)[:, None], sigma)
        moved = f(sub)
        worst = 0.0
        for cam in cams:
            a, _ = _pinhole(cam, sub)
            b, _ = _pinhole(cam, moved)
            worst = max(worst, float(np.abs(b - a).max()))
        if worst <= cap_px:
            break
        scale *= 0.97 * cap_px / worst
    f = _BodyField(centers, _axis_angle_quat(axes, angles * scale), tdir * (tmag * scale)[:, None], sigma)
    means = f(mu)
    q = _quat_mul(f.rotation(mu), scene.quats.astype(np.float64))
    q[q[:, 0] < 0] *= -1.0
    return Motion(means=means.astype(np.float32), quats=q.astype(np.float32),
                  scales=scene.scales.copy(), field=f)


# --------------------------------------------------------------------------
# proxy track fields
# --------------------------------------------------------------------------
def _surface_points(cam: Camera, radius, xs=None, ys=None):
    """First intersection of each pixel ray with the sphere |x| = radius
    (closest approach to the origin where the ray misses).  xs/ys select a
    lattice of pixel columns/rows (default: every pixel)."""
    xs = np.arange(cam.W, dtype=np.float64) if xs is None else np.asarray(xs, np.float64)
    ys = np.arange(cam.H, dtype=np.float64) if ys is None else np.asarray(ys, np.float64)
    cc, rr = np.meshgrid(xs, ys)
    dirc = np.stack([(cc - cam.cx) / cam.fx, (rr - cam.cy) / cam.fy, np.ones_like(cc)], -1)
    R = cam.R.astype(np.float64)
    dw = dirc @ R                    # camera -> world direction (R^T d)
    dw /= np.linalg.norm(dw, axis=-1, keepdims=True)
    o = cam.center
    b = dw @ o
    c = o @ o - radius * radius
    disc = b * b - c
    s_hit = -b - np.sqrt(np.maximum(disc, 0.0))
    s_far = -b
    s = np.where(disc > 0, s_hit, s_far)
    return o + dw * s[..., None]


def _lattice(n, stride):
    xs = np.arange(0, n, stride)
    if xs[-1] != n - 1:
        xs = np.append(xs, n - 1)
    return xs


def _lerp_axis(a, nodes, n, axis):
    """Linear interpolation of `a` sampled at `nodes` along `axis` to 0..n-1."""
    f = np.arange(n, dtype=np.float64)
    i0 = np.clip(np.searchsorted(nodes, f, side="right") - 1, 0, len(nodes) - 2)
    t = (f - nodes[i0]) / (nodes[i0 + 1] - nodes[i0])
    a0 = np.take(a, i0, axis=axis)
    a1 = np.take(a, i0 + 1, axis=axis)
    shape = [1] * a.ndim
    shape[axis] = n
    t = t.reshape(shape)
    return a0 * (1.0 - t) + a1 * t


def proxy_tracks(rng, cams, motion_fn, *, radius, noise_px=0.5, outlier_rate=0.0,
                 vis_rate=1.0, cap_px=None, stride=4):
    """disp[V,H,W,2] float32 and vis[V,H,W] uint8 for every first-frame pixel.

    The smooth ground-truth flow is evaluated on a lattice of every
    `stride`-th pixel and interpolated bilinearly; noise, outliers and
    visibility are drawn per pixel."""
    V = len(cams)
    H, W = cams[0].H, cams[0].W
    disp = np.empty((V, H, W, 2), np.float32)
    vis = np.empty((V, H, W), np.uint8)
    xs, ys = _lattice(W, stride), _lattice(H, stride)
    gx, gy = np.meshgrid(xs.astype(np.float64), ys.astype(np.float64))
    x0 = np.stack([gx, gy], -1)
    for v, cam in enumerate(cams):
        X = _surface_points(cam, radius, xs, ys)
        Xm = motion_fn(X.reshape(-1, 3)).reshape(X.shape)
        x1, _ = _pinhole(cam, Xm)
        dl = x1 - x0
        if cap_px is not None:
            m = np.linalg.norm(dl, axis=-1, keepdims=True)
            dl = np.where(m > cap_px, dl * (cap_px / np.maximum(m, 1e-30)), dl)
        d = _lerp_axis(_lerp_axis(dl, xs, W, 1), ys, H, 0).astype(np.float32)
        if noise_px > 0:
            d += rng.normal(0.0, noise_px, d.shape).astype(np.float32)
        if outlier_rate > 0:
            om = rng.random((H, W)) < outlier_rate
            k = int(om.sum())
            rr, cc = np.nonzero(om)
            d[rr, cc, 0] = (rng.uniform(0, W, k) - cc).astype(np.float32)
            d[rr, cc, 1] = (rng.uniform(0, H, k) - rr).astype(np.float32)
        disp[v] = d
        if vis_rate < 1.0:
            vis[v] = (rng.random((H, W)) < vis_rate).astype(np.uint8)
        else:
            vis[v] = 1
    return disp, vis


def _nearest_gaussian_motion(scene: Scene, motion: Motion):
    """Motion field for per-Gaussian motions: a point follows the rigid motion
    of its nearest Gaussian centre (proxy only)."""
    mu = scene.means.astype(np.float64)
    dq = _quat_mul(motion.quats.astype(np.float64),
                   scene.quats.astype(np.float64) * np.array([1, -1, -1, -1]))
    Rm = _quat_to_mat(dq)
    tm = motion.means.astype(np.float64)

    def fn(X):
        X = np.asarray(X, np.float64)
        out = np.empty_like(X)
        for s in range(0, X.shape[0], 4096):
            Xs = X[s:s + 4096]
            d2 = (Xs * Xs).sum(1)[:, None] - 2.0 * Xs @ mu.T + (mu * mu).sum(1)[None, :]
            k = np.argmin(d2, 1)
            out[s:s + 4096] = np.einsum("nij,nj->ni", Rm[k], Xs - mu[k]) + tm[k]
        return out
    return fn


# --------------------------------------------------------------------------
# named workloads (the paper-shaped configurations)
# --------------------------------------------------------------------------
WORKLOADS = {
    # 2k Gaussians in [-1,1]^3, 4 ring cameras at radius 3, 128x128
    "small": dict(n=2000, domain="cube", cams=("ring", 4, 3.0, 128, 128), motion="per_gaussian",
                  max_angle=10.0, max_trans=0.1, noise=0.5, outlier=0.0, vis=1.0, cap=None,
                  proxy_radius=1.2, seed=1),
    # 300k Gaussians in a radius-2 ball, 27 hemisphere cameras, 1352x1014
    "medium": dict(n=300_000, domain="ball", cams=("hemi", 27, 6.0, 1352, 1014), motion="bodies",
                   max_angle=10.0, max_trans=0.2, noise=1.0, outlier=0.0, vis=1.0, cap=60.0,
                   proxy_radius=2.0, seed=2),
    # 1M Gaussians, 20 hemisphere cameras, 1920x1080, large motions, outliers, visibility
    "large": dict(n=1_000_000, domain="ball", cams=("hemi", 20, 6.0, 1920, 1080), motion="bodies",
                  max_angle=30.0, max_trans=0.3, noise=1.0, outlier=0.05, vis=0.9, cap=150.0,
                  proxy_radius=2.0, seed=3),
}


def make_cameras(spec):
    kind, n, radius, W, H = spec
    if kind == "ring":
        return ring_cameras(n, radius, W, H)
    return hemisphere_cameras(n, radius, W, H)


def make_workload(name="small", *, seed=None, n=None, views=None, width=None, height=None,
                  with_tracks=True) -> Workload:
    """Build a named workload; size overrides shrink it for quick tests."""
    spec = dict(WORKLOADS[name])
    seed = spec["seed"] if seed is None else seed
    rng = np.random.default_rng(seed)
    kind, nv, rad, W, H = spec["cams"]
    nv = nv if views is None else views
    W = W if width is None else width
    H = H if height is None else height
    cams = make_cameras((kind, nv, rad, W, H))
    N = spec["n"] if n is None else n
    scene = random_gaussians(rng, N, domain=spec["domain"], radius=2.0)
    if spec["motion"] == "per_gaussian":
        motion = per_gaussian_rigid_motion(rng, scene, spec["max_angle"], spec["max_trans"])
        fn = _nearest_gaussian_motion(scene, motion)
    else:
        motion = body_field_motion(rng, scene, cams, max_angle_deg=spec["max_angle"],
                                   max_trans=spec["max_trans"], cap_px=spec["cap"])
        fn = motion.field
    if with_tracks:
        disp, vis = proxy_tracks(rng, cams, fn, radius=spec["proxy_radius"], noise_px=spec["noise"],
                                 outlier_rate=spec["outlier"], vis_rate=spec["vis"],
                                 cap_px=None if spec["cap"] is None else 1.25 * spec["cap"])
    else:
        disp = np.zeros((nv, H, W, 2), np.float32)
        vis = np.ones((nv, H, W), np.uint8)
    return Workload(name=name, scene=scene, cams=cams, motion=motion, disp=disp, vis=vis,
                    meta=dict(seed=seed, n=N, views=nv, W=W, H=H))


# --------------------------------------------------------------------------
# refinement workloads: ground-truth Gaussians with degree-3 SH colour and a
# perturbed copy to refine against images of the ground truth
# --------------------------------------------------------------------------
REFINE_WORKLOADS = {
    # gradient-check subset: 500 Gaussians, 64x64, two ring views
    "refine_fd": dict(n=500, domain="cube", cams=("ring", 2, 3.0, 64, 64), seed=11),
    # 500k Gaussians in a radius-2 ball, 16 hemisphere views at 1352x1014
    "refine": dict(n=500_000, domain="ball", cams=("hemi", 16, 6.0, 1352, 1014), seed=4),
}


@dataclass
class RefineWorkload:
    name: str
    gt: dict          # parameters of the ground truth (see refine_params)
    init: dict        # perturbed parameters the refinement starts from
    cams: list
    meta: dict


def refine_params(scene: Scene) -> dict:
    """Unconstrained parameters: means, quats, log-scales, opacity logits,
    SH coefficients [N, (deg+1)^2, 3]."""
    n = scene.n
    k = scene.sh.shape[1] // 3
    return dict(means=scene.means.astype(np.float32), quats=scene.quats.astype(np.float32),
                log_scales=np.log(scene.scales).astype(np.float32),
                logit_opacity=np.log(scene.opacity / (1.0 - scene.opacity)).astype(np.float32),
                sh=scene.sh.reshape(n, k, 3).astype(np.float32))


def make_refine_workload(name="refine", *, seed=None, n=None, views=None, width=None, height=None,
                         sigma_mean=0.01, sigma_log_scale=0.1, sigma_logit=0.2, sigma_sh=0.05,
                         sigma_quat=0.05) -> RefineWorkload:
    spec = dict(REFINE_WORKLOADS[name])
    seed = spec["seed"] if seed is None else seed
    rng = np.random.default_rng(seed)
    kind, nv, rad, W, H = spec["cams"]
    nv = nv if views is None else views
    W = W if width is None else width
    H = H if height is None else height
    cams = make_cameras((kind, nv, rad, W, H))
    N = spec["n"] if n is None else n
    scene = random_gaussians(rng, N, domain=spec["domain"], radius=2.0, sh_degree=3)
    gt = refine_params(scene)
    init = dict(
        means=(gt["means"] + rng.normal(0.0, sigma_mean, gt["means"].shape)).astype(np.float32),
        quats=(gt["quats"] + rng.normal(0.0, sigma_quat, gt["quats"].shape)).astype(np.float32),
        log_scales=(gt["log_scales"] + rng.normal(0.0, sigma_log_scale, gt["log_scales"].shape)).astype(np.float32),
        logit_opacity=(gt["logit_opacity"] + rng.normal(0.0, sigma_logit, N)).astype(np.float32),
        sh=(gt["sh"] + rng.normal(0.0, sigma_sh, gt["sh"].shape)).astype(np.float32))
    return RefineWorkload(name=name, gt=gt, init=init, cams=cams,
                          meta=dict(seed=seed, n=N, views=nv, W=W, H=H))


# --------------------------------------------------------------------------
# clips: a first frame's Gaussians plus F target frames of tracks (each
# target frame is tracked from the first frame; frame f carries the motion
# scaled to f / F, fresh noise, outliers and visibility)
# --------------------------------------------------------------------------
@dataclass
class Clip:
    name: str
    scene: Scene
    cams: list
    disp: np.ndarray          # [F,V,H,W,2] float32
    vis: np.ndarray           # [F,V,H,W] uint8
    meta: dict = field(default_factory=dict)


def make_clip(name="small", frames=3, *, seed=None, n=None, views=None, width=None, height=None) -> Clip:
    spec = dict(WORKLOADS[name])
    seed = spec["seed"] if seed is None else seed
    wl = make_workload(name, seed=seed, n=n, views=views, width=width, height=height, with_tracks=False)
    fn = wl.motion.field if wl.motion.field is not None else _nearest_gaussian_motion(wl.scene, wl.motion)
    rng = np.random.default_rng(seed + 7919)
    disp, vis = [], []
    for f in range(1, frames + 1):
        frac = f / frames

        def fn_f(X, frac=frac):
            return X + frac * (fn(X) - X)

        d, v = proxy_tracks(rng, wl.cams, fn_f, radius=spec["proxy_radius"], noise_px=spec["noise"],
                            outlier_rate=spec["outlier"], vis_rate=spec["vis"],
                            cap_px=None if spec["cap"] is None else 1.25 * spec["cap"])
        disp.append(d)
        vis.append(v)
    return Clip(name=name, scene=wl.scene, cams=wl.cams, disp=np.stack(disp), vis=np.stack(vis),
                meta=dict(wl.meta, frames=frames))


# --------------------------------------------------------------------------
# regularisation inputs: first-frame Gaussians, a multi-view update of them
# (a smooth rigid motion plus noise and salt-and-pepper outliers), the
# update's status bits and per-view pixel counts
# --------------------------------------------------------------------------
@dataclass
class RegCase:
    scene: Scene              # first frame
    means1: np.ndarray        # updated means [N,3]
    quats1: np.ndarray        # updated quaternions [N,4]
    scales1: np.ndarray       # updated scales [N,3]
    status: np.ndarray        # uint32 [N] (1 position, 2 covariance, other bits: reasons)
    acc: np.ndarray           # [V,N,16] float32, slots 12 (pixels) and 13 (static pixels) set
    truth: dict               # ground-truth motion: means, quats, scales


def make_reg_case(n=3000, views=4, *, seed=0, angle_deg=10.0, trans=0.1, noise=0.002, outlier_frac=0.05,
                  unsolved_frac=0.1, posonly_frac=0.05, static_frac=0.1, uniform=False, offset=None,
                  dup_frac=0.0, shell=None) -> RegCase:
    """Seeded regularisation input.  The options after `uniform` leave the
    base draws untouched: `offset` translates both frames (a scene far from
    the origin), `dup_frac` gives that fraction of Gaussians the first-frame
    position of another one (equal distances, ties by index), `shell` = r
    leaves only Gaussians farther than r from the ball's centre solved (the
    visible-surface pattern: an interior far from every solved Gaussian)."""
    rng = np.random.default_rng(seed)
    sc = random_gaussians(rng, n, domain="ball", radius=2.0)
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    qR = _axis_angle_quat(axis, math.radians(angle_deg))
    R = _quat_to_mat(qR)
    t = rng.standard_normal(3)
    t *= trans / np.linalg.norm(t)
    c = rng.uniform(-1.0, 1.0, 3)
    mu0 = sc.means.astype(np.float64)
    if uniform:
        # the same change for every Gaussian: translation plus a rotation of
        # each Gaussian about its own centre
        mu_t = mu0 + t
    else:
        mu_t = (mu0 - c) @ R.T + c + t
    q_t = np.stack([_quat_mul(qR, q) for q in sc.quats.astype(np.float64)])
    q_t[q_t[:, 0] < 0] *= -1.0
    s_t = sc.scales.astype(np.float64)
    truth = dict(means=mu_t, quats=q_t, scales=s_t)
    mu1 = mu_t + (0.0 if uniform else noise) * rng.standard_normal(mu_t.shape)
    q1 = q_t.copy()
    s1 = s_t * (1.0 + (0.0 if uniform else 0.01) * rng.standard_normal(s_t.shape))
    out = rng.random(n) < (0.0 if uniform else outlier_frac)
    mu1[out] += rng.normal(0.0, 0.5, (out.sum(), 3))
    q1[out] = _unit_quats(rng, out.sum())
    s1[out] *= rng.uniform(0.3, 3.0, (out.sum(), 3))
    status = np.full(n, 3, np.uint32)
    u = rng.random(n)
    status[u < unsolved_frac] = 4                                   # too few views
    status[(u >= unsolved_frac) & (u < unsolved_frac + posonly_frac)] = 1 | 32   # position only
    acc = np.zeros((views, n, 16), np.float32)
    acc[:, :, 12] = rng.integers(0, 40, (views, n))
    acc[:, :, 13] = np.floor(acc[:, :, 12] * rng.uniform(0.0, 0.5, (views, n)))
    st = rng.random(n) < static_frac
    for i in np.nonzero(st)[0]:
        vs = rng.choice(views, 2, replace=False)
        acc[vs, i, 12] = rng.integers(10, 40, 2)
        acc[vs, i, 13] = acc[vs, i, 12]
    rng2 = np.random.default_rng(seed + 7919)
    if dup_frac > 0.0:
        d = np.nonzero(rng2.random(n) < dup_frac)[0]
        src = rng2.integers(0, n, d.size)
        sc.means[d] = sc.means[src]
    if shell is not None:
        inner = np.linalg.norm(sc.means.astype(np.float64), axis=1) <= shell
        status[inner & (status == 3)] = 4
    if offset is not None:
        off = np.asarray(offset, np.float64)
        sc.means[:] = (sc.means.astype(np.float64) + off).astype(np.float32)
        mu1 = mu1 + off
        truth["means"] = truth["means"] + off
    return RegCase(scene=sc, means1=mu1.astype(np.float32), quats1=q1.astype(np.float32),
                   scales1=s1.astype(np.float32), status=status, acc=acc, truth=truth)
