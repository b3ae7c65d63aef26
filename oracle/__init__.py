"""CPU oracle for TrackerSplat motion transfer -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library: the only thing both
sides consume is the seeded input generator (`synth`), which holds none of the
method's arithmetic.

Contents, in the order the method runs (TrackerSplat, SIGGRAPH Asia 2025):

  geometry()       FP32 geometry decisions: splat centre, tile rectangle, depth
                   key, culling (Sec. 3.1, Eq. 1; the decisions are taken in the
                   renderer's FP32 precision; see tg_oracle.c).
  project64()      FP64 EWA covariance Sigma_2D = J W Sigma_3D W^T J^T and the
                   conic of its dilated form (Sec. 3.1, Eq. 1).
  cell_lists()     brute-force depth-ordered per-tile lists (Sec. 3.1: the
                   splats are blended front to back by depth).
  composite()      per-pixel compositing with w = alpha*T and the weighted
                   incremental LS statistics (Sec. 4.3.3, Sec. 4.3.4 Eq. 4).
  solve_views()    [A|b] per (Gaussian, view) from V1^{-1} V2 and Eq. 2
                   (Sec. 4.2 Eq. 2, Sec. 4.3.4, thresholds of Sec. 5.2).
  triangulate()    multi-view update: SVD triangulation of the mean, the
                   6-unknown covariance system, eigendecomposition with reorder
                   (Sec. 4.4.1-4.4.3, thresholds of Sec. 5.2).
  motion_transfer() the steps above end to end.

Readings where the paper is silent or ambiguous are listed in the
repository's design notes; the constants below are those readings.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

# ---- constants (renderer readings; Sec. 5.2 thresholds) -------------------
TILE = 16
NEAR = 0.2
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
DET_MIN = 1e-12          # Sec. 5.2: V1 determinant below 1e-12 -> unsolvable
ISO_MIN = 1e-4           # near-singular V1 (Sec. 4.3.5), scale-invariant reading:
                         # covered pixels (nearly) on one line
WSUM_MIN = 1e-3          # Sec. 5.2: accumulated alpha below 1e-3 -> unsolvable
PIX_MIN = 2              # Sec. 5.2: fewer than 2 pixels -> unsolvable
VIEWS_MIN = 2            # Sec. 5.2: visible in fewer than 2 views
WSUM_TOTAL_MIN = 1e-3    # Sec. 5.2: accumulated alpha across views
PIX_TOTAL_MIN = 3        # Sec. 5.2: fewer than 3 pixels across views
JCLAMP = 1.3

# per-view flags
VF_OK, VF_CULLED, VF_FEW_PIX, VF_LOW_ALPHA, VF_SINGULAR, VF_NONFINITE = 1, 2, 4, 8, 16, 32
# per-Gaussian status bits
ST_POS, ST_COV, ST_FEW_VIEWS, ST_LOW_ALPHA, ST_FEW_PIX = 1, 2, 4, 8, 16
ST_NEG_EIG, ST_DLT_DEGEN, ST_BEHIND, ST_NONFINITE = 32, 64, 128, 256

# accumulator record slots
S_W, S_UX, S_UY, S_UXUX, S_UXUY, S_UYUY, S_DX, S_DY = range(8)
S_UXDX, S_UXDY, S_UYDX, S_UYDY, S_N, S_STATN, S_STATA = range(8, 15)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_geometry_f32.argtypes = [i64, P, P, P, i32, P, P, P, P, P]
        L.orc_geometry_f32.restype = None
        L.orc_project_f64.argtypes = [i64, P, P, P, i32, P, P, P]
        L.orc_project_f64.restype = None
        L.orc_tile_lists.argtypes = [i64, i32, P, P, P, P, i32, P, P, i64]
        L.orc_tile_lists.restype = i64
        L.orc_composite.argtypes = [i32, P, i64, P, P, P, P, P, P, P, P, f64, f64,
                                    P, P, P, P, P, P, P, P]
        L.orc_composite.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = i32
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        _lib = L
    return _lib


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def cam_array(cams):
    return np.ascontiguousarray(synth.camera_array(cams))


# ---------------------------------------------------------------------------
@dataclass
class Geometry:
    mu: np.ndarray      # [V,N,2] float32 splat centre
    rect: np.ndarray    # [V,N,4] int32 (tx0, ty0, tx1, ty1)
    key: np.ndarray     # [V,N] uint32 depth key (FP32 bits of p_z)
    valid: np.ndarray   # [V,N] uint8


def geometry(scene, cams) -> Geometry:
    N, V = scene.n, len(cams)
    ca = cam_array(cams)
    mu = np.zeros((V, N, 2), np.float32)
    rect = np.zeros((V, N, 4), np.int32)
    key = np.zeros((V, N), np.uint32)
    valid = np.zeros((V, N), np.uint8)
    m, q, s = _c(scene.means, np.float32), _c(scene.quats, np.float32), _c(scene.scales, np.float32)
    lib().orc_geometry_f32(N, _p(m), _p(q), _p(s), V, _p(ca), _p(mu), _p(rect), _p(key), _p(valid))
    # a Gaussian with a non-finite parameter is culled in every view
    bad = ~finite_params(scene)
    if bad.any():
        mu[:, bad] = 0.0
        rect[:, bad] = 0
        key[:, bad] = 0xFFFFFFFF
        valid[:, bad] = 0
    return Geometry(mu, rect, key, valid)


def finite_params(scene):
    """[N] bool: mean, quaternion, scale and opacity all finite."""
    return (np.isfinite(scene.means).all(1) & np.isfinite(scene.quats).all(1) &
            np.isfinite(scene.scales).all(1) & np.isfinite(scene.opacity))


def project64(scene, cams):
    """FP64 (undilated Sigma_2D, conic of the dilated Sigma_2D), each [V,N,3]."""
    N, V = scene.n, len(cams)
    ca = cam_array(cams)
    cov = np.zeros((V, N, 3), np.float64)
    conic = np.zeros((V, N, 3), np.float64)
    m, q, s = _c(scene.means, np.float32), _c(scene.quats, np.float32), _c(scene.scales, np.float32)
    lib().orc_project_f64(N, _p(m), _p(q), _p(s), V, _p(ca), _p(cov), _p(conic))
    return cov, conic


def depth_order(geom: Geometry):
    """Per view: indices of the non-culled Gaussians sorted by (key, index)."""
    out = []
    for v in range(geom.key.shape[0]):
        idx = np.nonzero(geom.valid[v])[0]
        k = geom.key[v, idx]
        out.append(idx[np.lexsort((idx, k))].astype(np.uint32))
    return out


def cell_lists(geom: Geometry, cams, cell=1):
    """CSR (starts[int64, n_cells+1], ids[uint32]) over all views' cells of
    cell x cell tiles, row-major per view, views concatenated."""
    V, N = geom.key.shape
    ca = cam_array(cams)
    ncell = 0
    for c in cams:
        TX, TY = -(-c.W // TILE), -(-c.H // TILE)
        ncell += (-(-TX // cell)) * (-(-TY // cell))
    starts = np.zeros(ncell + 1, np.int64)
    L = lib()
    tot = L.orc_tile_lists(N, V, _p(ca), _p(geom.rect), _p(geom.key), _p(geom.valid), cell,
                           _p(starts), None, 0)
    ids = np.zeros(max(int(tot), 1), np.uint32)
    r = L.orc_tile_lists(N, V, _p(ca), _p(geom.rect), _p(geom.key), _p(geom.valid), cell,
                         _p(starts), _p(ids), ids.size)
    assert r == tot
    return starts, ids[:tot]


def composite(scene, cams, geom: Geometry, conic, lists, disp, vis=None, pixmask=None,
              raw=False, band_alpha=1e-5, band_t=2e-5):
    """Depth-ordered compositing with the PWI-LS statistics (FP64).

    Returns dict with mom/absm/slack [V,N,16], nmarg [V,N], raw [V,N,15]
    (optional), tfinal [V,H,W], pixmarg [V,H,W], counters [V,2]
    (evaluated pairs, contributing pairs)."""
    V, N = geom.key.shape
    H, W = cams[0].H, cams[0].W
    ca = cam_array(cams)
    starts, ids = lists
    mom = np.zeros((V, N, 16), np.float64)
    absm = np.zeros((V, N, 16), np.float64)
    slack = np.zeros((V, N, 16), np.float64)
    nmarg = np.zeros((V, N), np.int32)
    rawa = np.zeros((V, N, 15), np.float64) if raw else None
    tfinal = np.ones((V, H, W), np.float64)
    pixmarg = np.zeros((V, H, W), np.uint8)
    counters = np.zeros((V, 2), np.int64)
    d = _c(disp, np.float32)
    vv = None if vis is None else _c(vis, np.uint8)
    pm = None if pixmask is None else _c(pixmask, np.uint8)
    op = _c(scene.opacity, np.float32)
    conic = _c(conic, np.float64)
    lib().orc_composite(V, _p(ca), N, _p(geom.mu), _p(conic), _p(op), _p(starts), _p(ids),
                        _p(d), _p(vv), _p(pm), band_alpha, band_t, _p(mom), _p(absm), _p(slack),
                        _p(nmarg), _p(rawa), _p(tfinal), _p(pixmarg), _p(counters))
    return dict(mom=mom, absm=absm, slack=slack, nmarg=nmarg, raw=rawa, tfinal=tfinal,
                pixmarg=pixmarg, counters=counters)


# ---------------------------------------------------------------------------
# per-view solve (Sec. 4.3.4 Eq. 4 with the Sec. 5.2 thresholds; Sec. 4.2 Eq. 2)
# ---------------------------------------------------------------------------
def v1_v2(mom):
    """Centred V1 (3x3) and V2 (3x2) from accumulator records [...,16]."""
    m = mom
    V1 = np.empty(m.shape[:-1] + (3, 3))
    V1[..., 0, 0], V1[..., 0, 1], V1[..., 0, 2] = m[..., S_UXUX], m[..., S_UXUY], m[..., S_UX]
    V1[..., 1, 0], V1[..., 1, 1], V1[..., 1, 2] = m[..., S_UXUY], m[..., S_UYUY], m[..., S_UY]
    V1[..., 2, 0], V1[..., 2, 1], V1[..., 2, 2] = m[..., S_UX], m[..., S_UY], m[..., S_W]
    V2 = np.empty(m.shape[:-1] + (3, 2))
    V2[..., 0, 0], V2[..., 0, 1] = m[..., S_UXDX], m[..., S_UXDY]
    V2[..., 1, 0], V2[..., 1, 1] = m[..., S_UYDX], m[..., S_UYDY]
    V2[..., 2, 0], V2[..., 2, 1] = m[..., S_DX], m[..., S_DY]
    return V1, V2


def solve_views(mom, mu_c, cov, rendered):
    """Per (view, Gaussian): flags, new 2D mean and covariance (Eq. 2).

    The LS regresses the displacement dd = x' - x on [u; 1], u = x - mu_c,
    which is the paper's x' = A x + b re-parametrised (exact in real
    arithmetic): Theta = V1^{-1} V2 = [G^T; c^T], A = I + G,
    mu' = mu_c + c, Sigma' = A Sigma A^T.  Unsolved entries keep A = I,
    c = 0 and get zero mu' and Sigma'."""
    V, N = mom.shape[:2]
    V1, V2 = v1_v2(mom)
    det = np.linalg.det(V1)
    flags = np.zeros((V, N), np.uint8)
    flags |= np.where(rendered == 0, VF_CULLED, 0).astype(np.uint8)
    flags |= np.where(mom[..., S_N] < PIX_MIN, VF_FEW_PIX, 0).astype(np.uint8)
    flags |= np.where(mom[..., S_W] < WSUM_MIN, VF_LOW_ALPHA, 0).astype(np.uint8)
    flags |= np.where(~(det >= DET_MIN), VF_SINGULAR, 0).astype(np.uint8)
    # a non-finite track leaves non-finite sums in the record
    flags |= np.where(~np.isfinite(mom[..., :13]).all(-1), VF_NONFINITE, 0).astype(np.uint8)
    # weighted covariance C of the pixel offsets u; near-singular when
    # 4 det(C) / tr(C)^2 < ISO_MIN (its eigenvalues differ by ~1/ISO_MIN)
    with np.errstate(divide="ignore", invalid="ignore"):
        sw = mom[..., S_W]
        mx, my = mom[..., S_UX] / sw, mom[..., S_UY] / sw
        ca = mom[..., S_UXUX] / sw - mx * mx
        cb = mom[..., S_UXUY] / sw - mx * my
        cc = mom[..., S_UYUY] / sw - my * my
        tr = ca + cc
        iso_ok = (tr > 0) & (4.0 * (ca * cc - cb * cb) >= ISO_MIN * tr * tr)
    flags |= np.where(~iso_ok, VF_SINGULAR, 0).astype(np.uint8)
    ok = flags == 0
    flags[ok] = VF_OK
    A = np.zeros((V, N, 2, 2))
    A[..., 0, 0] = A[..., 1, 1] = 1.0
    c = np.zeros((V, N, 2))
    mu_new = np.zeros((V, N, 2))
    cov_new = np.zeros((V, N, 3))
    if ok.any():
        theta = np.linalg.solve(V1[ok], V2[ok])               # [n,3,2]
        Ak = np.eye(2) + np.swapaxes(theta[:, 0:2, :], -1, -2)
        ck = theta[:, 2, :]
        S = cov[ok]
        Sk = np.empty((S.shape[0], 2, 2))
        Sk[:, 0, 0], Sk[:, 0, 1], Sk[:, 1, 0], Sk[:, 1, 1] = S[:, 0], S[:, 1], S[:, 1], S[:, 2]
        Sn = Ak @ Sk @ np.swapaxes(Ak, -1, -2)
        A[ok] = Ak
        c[ok] = ck
        mu_new[ok] = np.asarray(mu_c, np.float64)[ok] + ck
        cov_new[ok] = np.stack([Sn[:, 0, 0], Sn[:, 0, 1], Sn[:, 1, 1]], -1)
    return dict(flags=flags, mu_new=mu_new, cov_new=cov_new, A=A, c=c, det=det)


# ---------------------------------------------------------------------------
# multi-view update (Sec. 4.4.1-4.4.3)
# ---------------------------------------------------------------------------
def quat_to_rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = np.moveaxis(q, -1, 0)
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def rot_to_quat(R):
    """Rotation matrix -> unit quaternion (w,x,y,z), w >= 0 (Shepperd's
    method: pivot on the largest of w^2, x^2, y^2, z^2)."""
    R = np.asarray(R, np.float64)
    tr = R[..., 0, 0] + R[..., 1, 1] + R[..., 2, 2]
    cand = np.stack([tr, R[..., 0, 0], R[..., 1, 1], R[..., 2, 2]], -1)
    k = np.argmax(cand, -1)
    q = np.zeros(R.shape[:-2] + (4,))
    r = R
    # case w
    s = np.sqrt(np.maximum(1 + tr, 0)) * 2
    qw = np.stack([0.25 * s, (r[..., 2, 1] - r[..., 1, 2]) / s, (r[..., 0, 2] - r[..., 2, 0]) / s,
                   (r[..., 1, 0] - r[..., 0, 1]) / s], -1)
    s = np.sqrt(np.maximum(1 + r[..., 0, 0] - r[..., 1, 1] - r[..., 2, 2], 0)) * 2
    qx = np.stack([(r[..., 2, 1] - r[..., 1, 2]) / s, 0.25 * s, (r[..., 0, 1] + r[..., 1, 0]) / s,
                   (r[..., 0, 2] + r[..., 2, 0]) / s], -1)
    s = np.sqrt(np.maximum(1 - r[..., 0, 0] + r[..., 1, 1] - r[..., 2, 2], 0)) * 2
    qy = np.stack([(r[..., 0, 2] - r[..., 2, 0]) / s, (r[..., 0, 1] + r[..., 1, 0]) / s, 0.25 * s,
                   (r[..., 1, 2] + r[..., 2, 1]) / s], -1)
    s = np.sqrt(np.maximum(1 - r[..., 0, 0] - r[..., 1, 1] + r[..., 2, 2], 0)) * 2
    qz = np.stack([(r[..., 1, 0] - r[..., 0, 1]) / s, (r[..., 0, 2] + r[..., 2, 0]) / s,
                   (r[..., 1, 2] + r[..., 2, 1]) / s, 0.25 * s], -1)
    with np.errstate(invalid="ignore", divide="ignore"):
        q = np.where((k == 0)[..., None], qw, np.where((k == 1)[..., None], qx,
                     np.where((k == 2)[..., None], qy, qz)))
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    q = np.where((q[..., 0] < 0)[..., None], -q, q)
    return q


def _cam_mats(cams):
    R = np.stack([c.R.astype(np.float64) for c in cams])
    t = np.stack([c.t.astype(np.float64) for c in cams])
    K = np.array([[np.float64(np.float32(c.fx)), np.float64(np.float32(c.fy)),
                   np.float64(np.float32(c.cx)), np.float64(np.float32(c.cy)),
                   c.W, c.H] for c in cams])
    return R, t, K


def cov_rows(cams, mu3):
    """Rows of the linear system Sigma_2D' = J W Sigma_3D' W^T J^T (Sec. 4.4.2)
    for every view at the 3D means mu3 [N,3]: returns [V,N,3,6]; unknown order
    (S00, S01, S02, S11, S12, S22), rows for the (0,0), (0,1), (1,1) entries."""
    R, t, K = _cam_mats(cams)
    p = np.einsum("vij,nj->vni", R, mu3) + t[:, None, :]
    pz = p[..., 2]
    fx, fy = K[:, 0][:, None], K[:, 1][:, None]
    limx = JCLAMP * (0.5 * K[:, 4] / K[:, 0])[:, None]
    limy = JCLAMP * (0.5 * K[:, 5] / K[:, 1])[:, None]
    tx = np.clip(p[..., 0] / pz, -limx, limx)
    ty = np.clip(p[..., 1] / pz, -limy, limy)
    V, N = pz.shape
    J = np.zeros((V, N, 2, 3))
    J[..., 0, 0] = fx / pz
    J[..., 0, 2] = -fx * tx / pz
    J[..., 1, 1] = fy / pz
    J[..., 1, 2] = -fy * ty / pz
    T = J @ R[:, None, :, :]
    rows = []
    for a, b in ((0, 0), (0, 1), (1, 1)):
        Ta, Tb = T[..., a, :], T[..., b, :]
        rows.append(np.stack([Ta[..., 0] * Tb[..., 0],
                              Ta[..., 0] * Tb[..., 1] + Ta[..., 1] * Tb[..., 0],
                              Ta[..., 0] * Tb[..., 2] + Ta[..., 2] * Tb[..., 0],
                              Ta[..., 1] * Tb[..., 1],
                              Ta[..., 1] * Tb[..., 2] + Ta[..., 2] * Tb[..., 1],
                              Ta[..., 2] * Tb[..., 2]], -1))
    return np.stack(rows, -2), pz


def dlt_rows(cams, mu2):
    """Homogeneous DLT rows (Sec. 4.4.1) in K^{-1}-normalised coordinates:
    [V,N,2,4] for 2D points mu2 [V,N,2]."""
    R, t, K = _cam_mats(cams)
    P = np.concatenate([R, t[:, :, None]], -1)           # [V,3,4]
    xn = (mu2[..., 0] - K[:, 2][:, None]) / K[:, 0][:, None]
    yn = (mu2[..., 1] - K[:, 3][:, None]) / K[:, 1][:, None]
    r1 = xn[..., None] * P[:, None, 2, :] - P[:, None, 0, :]
    r2 = yn[..., None] * P[:, None, 2, :] - P[:, None, 1, :]
    return np.stack([r1, r2], -2)


def triangulate(scene, cams, sv, mom, rendered, chunk=65536):
    """Multi-view update of mean, rotation and scale (Sec. 4.4)."""
    V, N = sv["flags"].shape
    ok = sv["flags"] == VF_OK
    nv = ok.sum(0)
    sw_tot = (mom[..., S_W] * (rendered != 0)).sum(0)
    n_tot = (mom[..., S_N] * (rendered != 0)).sum(0)
    status = np.zeros(N, np.uint32)
    # non-finite input: the Gaussian's own parameters, or a view's statistics
    nonfinite = ~finite_params(scene) | ((sv["flags"] & VF_NONFINITE) > 0).any(0)
    status |= np.where(nonfinite, ST_NONFINITE, 0).astype(np.uint32)
    status |= np.where(nv < VIEWS_MIN, ST_FEW_VIEWS, 0).astype(np.uint32)
    status |= np.where(~(sw_tot >= WSUM_TOTAL_MIN), ST_LOW_ALPHA, 0).astype(np.uint32)
    status |= np.where(n_tot < PIX_TOTAL_MIN, ST_FEW_PIX, 0).astype(np.uint32)
    means = scene.means.astype(np.float64).copy()
    quats = scene.quats.astype(np.float64).copy()
    scales = scene.scales.astype(np.float64).copy()
    R_old = quat_to_rot(quats)
    eig = np.zeros((N, 3))
    for s in range(0, N, chunk):
        e = min(N, s + chunk)
        cand = (status[s:e] & ~np.uint32(ST_NONFINITE)) == 0
        if not cand.any():
            continue
        idx = np.nonzero(cand)[0] + s
        okc = ok[:, idx]                                     # [V,n]
        rows = dlt_rows(cams, sv["mu_new"][:, idx])          # [V,n,2,4]
        rows = rows * okc[..., None, None]
        M = np.transpose(rows, (1, 0, 2, 3)).reshape(len(idx), 2 * V, 4)
        _, _, vh = np.linalg.svd(M)
        h = vh[:, -1, :]
        h = h / np.linalg.norm(h, axis=-1, keepdims=True)
        degen = np.abs(h[:, 3]) < 1e-12
        with np.errstate(divide="ignore", invalid="ignore"):
            mu3 = h[:, :3] / h[:, 3:4]
        mu3 = np.where(degen[:, None], 0.0, mu3)
        crows, pz = cov_rows(cams, mu3)                      # [V,n,3,6], [V,n]
        behind = ((pz <= NEAR) & okc).any(0)
        st = np.zeros(len(idx), np.uint32)
        st |= np.where(degen, ST_DLT_DEGEN, 0).astype(np.uint32)
        st |= np.where(behind & ~degen, ST_BEHIND, 0).astype(np.uint32)
        pos_ok = st == 0
        means[idx[pos_ok]] = mu3[pos_ok]
        st |= np.where(pos_ok, ST_POS, 0).astype(np.uint32)
        # covariance least squares, unweighted, valid views only
        A = np.transpose(crows * okc[..., None, None], (1, 0, 2, 3)).reshape(len(idx), 3 * V, 6)
        b = np.transpose(sv["cov_new"][:, idx] * okc[..., None], (1, 0, 2)).reshape(len(idx), 3 * V)
        sol = np.zeros((len(idx), 6))
        if pos_ok.any():
            sol[pos_ok] = np.einsum("nij,nj->ni", np.linalg.pinv(A[pos_ok], rcond=1e-13), b[pos_ok])
            sing = np.linalg.svd(A[pos_ok], compute_uv=False)
            rankdef = sing[:, -1] <= 1e-13 * sing[:, 0]
        Sg = np.stack([np.stack([sol[:, 0], sol[:, 1], sol[:, 2]], -1),
                       np.stack([sol[:, 1], sol[:, 3], sol[:, 4]], -1),
                       np.stack([sol[:, 2], sol[:, 4], sol[:, 5]], -1)], -2)
        lam, vec = np.linalg.eigh(Sg)                        # ascending
        negeig = pos_ok & ~(lam[:, 0] > 0)
        if pos_ok.any():
            rd = np.zeros(len(idx), bool)
            rd[pos_ok] = rankdef
            negeig |= rd
        st |= np.where(negeig, ST_NEG_EIG, 0).astype(np.uint32)
        cov_ok = pos_ok & ~negeig
        if cov_ok.any():
            ii = idx[cov_ok]
            so = scales[ii]
            rank_old = np.argsort(np.argsort(so, axis=1, kind="stable"), axis=1, kind="stable")
            vc = vec[cov_ok]
            lc = lam[cov_ok]
            Rn = np.take_along_axis(vc, rank_old[:, None, :].repeat(3, 1), axis=2)
            sn = np.sqrt(np.take_along_axis(lc, rank_old, axis=1))
            Ro = R_old[ii]
            dots = np.einsum("nik,nik->nk", Rn, Ro)
            Rn = Rn * np.where(dots < 0, -1.0, 1.0)[:, None, :]
            dots = np.abs(dots)
            neg = np.linalg.det(Rn) < 0
            kmin = np.argmin(dots, axis=1)
            flip = np.ones((len(ii), 3))
            flip[np.arange(len(ii)), kmin] = np.where(neg, -1.0, 1.0)
            Rn = Rn * flip[:, None, :]
            quats[ii] = rot_to_quat(Rn)
            scales[ii] = sn
            eig[ii] = lc
        st |= np.where(cov_ok, ST_COV, 0).astype(np.uint32)
        status[idx] |= st
    return dict(means=means, quats=quats, scales=scales, status=status, eig=eig)


# ---------------------------------------------------------------------------
def motion_transfer(scene, cams, disp, vis=None, raw=False, pixmask=None):
    geom = geometry(scene, cams)
    cov, conic = project64(scene, cams)
    lists = cell_lists(geom, cams, 1)
    comp = composite(scene, cams, geom, conic, lists, disp, vis, pixmask=pixmask, raw=raw)
    sv = solve_views(comp["mom"], geom.mu, cov, geom.valid)
    tri = triangulate(scene, cams, sv, comp["mom"], geom.valid)
    return dict(geom=geom, cov=cov, conic=conic, lists=lists, comp=comp, sv=sv, tri=tri)
