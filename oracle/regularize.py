"""Motion regularisation (Sec. 4.5) -- TEST INFRASTRUCTURE ONLY.

Plain numpy/scipy, FP64.  Steps in the paper's order:

  static_mask()   Sec. 4.5.2: a Gaussian counts as static when at least two
                  of its views each see it with ten or more covering pixels,
                  over nine tenths of them static (|x' - x| < 1 px; counted
                  by the accumulation, slots S_N and S_STATN).  Static
                  Gaussians keep their first-frame parameters and take no
                  further part.
  deltas()        Sec. 4.5.1: the change of a Gaussian against the first
                  frame: d_mu = mu' - mu, d_S = s' - s (linear scales) and
                  the rotation change Q = R' R^T in Euler-angle form
                  (Q = Rz(psi) Ry(theta) Rx(phi), angles (phi, theta, psi)).
  knn()           the K = 8 nearest solved Gaussians (Sec. 5.2), by the
                  Euclidean distance between first-frame means; a solved
                  Gaussian's own entry is among them (distance 0).
  median_filter() Sec. 4.5.1: a solved Gaussian takes the component-wise
                  median of its neighbours' changes.
  propagate()     Sec. 4.5.2: a Gaussian that is neither solved nor static
                  takes the component-wise mean of its neighbours' filtered
                  changes.
  regularize()    the steps above; the change is added to the first-frame
                  parameters (rotation: R_new = Q(angles) R).

"Solved" means position and covariance both updated by the multi-view step
(status bits 1 and 2); Gaussians with only a position (negative eigenvalue
or singular covariance system) are propagation targets, as the paper names
negative eigenvalues among the unreliable cases.  A scale component that
would become non-positive keeps its first-frame value.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import S_N, S_STATN, ST_COV, ST_POS, quat_to_rot, rot_to_quat

K = 8                 # neighbours (Sec. 5.2)
STATIC_MIN_PIX = 9    # static in a view: pixel count must exceed this (Sec. 4.5.2)
STATIC_FRAC = 0.9     # ... and the static share of them must exceed this
STATIC_VIEWS = 2      # static Gaussian: static in at least this many views

RG_STATIC, RG_FILTERED, RG_PROPAGATED = 1, 2, 4


def static_mask(acc):
    """acc [V,N,16] accumulator records -> bool [N]."""
    n = acc[..., S_N].astype(np.float64)
    sn = acc[..., S_STATN].astype(np.float64)
    per_view = (n > STATIC_MIN_PIX) & (sn > STATIC_FRAC * n)
    return per_view.sum(0) >= STATIC_VIEWS


def euler_zyx(Q):
    """Q = Rz(psi) Ry(theta) Rx(phi) -> (phi, theta, psi)."""
    theta = np.arcsin(np.clip(-Q[..., 2, 0], -1.0, 1.0))
    phi = np.arctan2(Q[..., 2, 1], Q[..., 2, 2])
    psi = np.arctan2(Q[..., 1, 0], Q[..., 0, 0])
    return np.stack([phi, theta, psi], -1)


def rot_zyx(e):
    """(phi, theta, psi) -> Rz(psi) Ry(theta) Rx(phi)."""
    phi, theta, psi = np.moveaxis(np.asarray(e, np.float64), -1, 0)
    cx, sx, cy, sy, cz, sz = np.cos(phi), np.sin(phi), np.cos(theta), np.sin(theta), np.cos(psi), np.sin(psi)
    Rx = np.stack([np.stack([np.ones_like(cx), 0 * cx, 0 * cx], -1), np.stack([0 * cx, cx, -sx], -1),
                   np.stack([0 * cx, sx, cx], -1)], -2)
    Ry = np.stack([np.stack([cy, 0 * cy, sy], -1), np.stack([0 * cy, np.ones_like(cy), 0 * cy], -1),
                   np.stack([-sy, 0 * cy, cy], -1)], -2)
    Rz = np.stack([np.stack([cz, -sz, 0 * cz], -1), np.stack([sz, cz, 0 * cz], -1),
                   np.stack([0 * cz, 0 * cz, np.ones_like(cz)], -1)], -2)
    return Rz @ Ry @ Rx


def deltas(means0, quats0, scales0, means1, quats1, scales1):
    """[N,9]: d_mu (3), Euler angles of R' R^T (3), d_S (3)."""
    R0 = quat_to_rot(quats0)
    R1 = quat_to_rot(quats1)
    d = np.zeros((means0.shape[0], 9))
    d[:, 0:3] = np.asarray(means1, np.float64) - np.asarray(means0, np.float64)
    d[:, 3:6] = euler_zyx(R1 @ np.swapaxes(R0, -1, -2))
    d[:, 6:9] = np.asarray(scales1, np.float64) - np.asarray(scales0, np.float64)
    return d


def knn(points, sources, queries, k=K):
    """Indices (into `sources`, ascending Gaussian indices) of the
    min(k, |sources|) nearest sources of each query point, nearest first,
    and their distances.  Equal distances are ordered by index (the paper
    does not say; the reading is that of the neighbourhood row of the design
    notes): the tree's candidates are re-sorted by (distance, index), and a
    query whose candidates all tie with its k-th is decided over all
    sources."""
    pts = np.asarray(points, np.float64)
    sources = np.asarray(sources)
    kk = min(k, len(sources))
    if kk == 0:
        return np.zeros((len(queries), 0), np.int64), np.zeros((len(queries), 0))
    tree = cKDTree(pts[sources])
    extra = min(len(sources), kk + 8)
    qp = pts[queries]
    _, idx = tree.query(qp, k=extra)
    if extra == 1:
        idx = idx[:, None]
    # squared distances of the candidates (the order is decided on these)
    d2 = ((pts[sources][idx] - qp[:, None, :]) ** 2).sum(-1)
    order = np.lexsort((idx, d2))            # per row: by distance, then index
    d2 = np.take_along_axis(d2, order, 1)
    idx = np.take_along_axis(idx, order, 1)
    # ties may reach past the fetched candidates: decide those rows over all sources
    open_rows = np.nonzero((extra < len(sources)) & (d2[:, extra - 1] == d2[:, kk - 1]))[0]
    for r in open_rows:
        d = ((pts[sources] - qp[r]) ** 2).sum(1)
        o = np.lexsort((np.arange(len(sources)), d))[:extra]
        d2[r], idx[r] = d[o], o
    return idx[:, :kk], np.sqrt(d2[:, :kk])


def median_filter(vals):
    """[n, K, 9] neighbours' changes (own entry first) -> [n, 9] (Sec. 4.5.1)."""
    return np.median(vals, axis=1)


def propagate(vals):
    """[n, K, 9] neighbours' filtered changes -> [n, 9] (Sec. 4.5.2)."""
    return vals.mean(axis=1)


def regularize(means0, quats0, scales0, means1, quats1, scales1, status, acc, k=None):
    """Returns (means, quats, scales, reg_status) after Sec. 4.5; k defaults
    to the module's K."""
    k = K if k is None else k
    N = means0.shape[0]
    status = np.asarray(status, np.uint32)
    static = static_mask(acc)
    solved = ((status & ST_POS) > 0) & ((status & ST_COV) > 0) & ~static
    d = deltas(means0, quats0, scales0, means1, quats1, scales1)
    out_d = np.zeros((N, 9))
    reg = np.where(static, RG_STATIC, 0).astype(np.uint32)
    src = np.nonzero(solved)[0]
    if src.size:
        # median filter of the solved Gaussians
        idx, _ = knn(means0, src, src, k)
        filt = median_filter(d[src][idx])                     # [n_src, 9]
        out_d[src] = filt
        reg[src] |= RG_FILTERED
        # propagation of the filtered changes to the rest (not static)
        tgt = np.nonzero(~solved & ~static)[0]
        if tgt.size:
            fd = np.zeros((N, 9))
            fd[src] = filt
            idx, _ = knn(means0, src, tgt, k)
            out_d[tgt] = propagate(fd[src][idx])
            reg[tgt] |= RG_PROPAGATED
    moved = (reg & (RG_FILTERED | RG_PROPAGATED)) > 0
    means = np.asarray(means0, np.float64).copy()
    quats = np.asarray(quats0, np.float64).copy()
    scales = np.asarray(scales0, np.float64).copy()
    means[moved] += out_d[moved, 0:3]
    R = rot_zyx(out_d[moved, 3:6]) @ quat_to_rot(quats0[moved])
    quats[moved] = rot_to_quat(R)
    s_new = scales[moved] + out_d[moved, 6:9]
    scales[moved] = np.where(s_new > 0, s_new, scales[moved])
    return means, quats, scales, reg
