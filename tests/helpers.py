"""Shared helpers for the GPU parity tests (HIP path vs the CPU oracle).

Inputs come from `synth` only; expected values from `oracle` only.
"""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle
import synth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(wl, capacity=None, t_final=True, stats=True, params=None, vis=True, disp=None):
    """Cold frame on the GPU; returns a dict of host arrays."""
    import torch
    from paper_2604_02586_amd import api
    dev = torch.device("cuda:0")
    g = api.GaussianTensors.from_scene(wl.scene, dev)
    mt = api.MotionTransfer(wl.cams, wl.scene.n, dev, params=params, capacity=capacity)
    d = torch.as_tensor(wl.disp if disp is None else disp).to(dev).contiguous()
    vv = torch.as_tensor(wl.vis).to(dev).contiguous() if vis else None
    out = mt.run(g, d, vv, t_final=t_final, stats=stats)
    torch.cuda.synchronize()
    h = lambda t: t.detach().cpu().numpy()
    res = dict(mt=mt, rec=h(mt.splats.rec), cov2d=h(mt.splats.cov2d),
                rect=h(mt.splats.rect).view(np.uint16), key=h(mt.splats.key).view(np.uint32),
                order=h(mt.bins.order).view(np.uint32), cell_ids=h(mt.bins.cell_ids).view(np.uint32),
                cell_ranges=h(mt.bins.cell_ranges).view(np.uint32), n_pairs=int(mt.bins.n_pairs.item()),
                overflow=int(mt.bins.overflow.item()), acc=h(mt.acc),
                t_final=h(mt.t_final) if t_final else None, stats=h(mt.stats),
                mu_new=h(mt.mu_new), cov_new=h(mt.cov_new), vflags=h(mt.vflags),
                status=h(mt.status).view(np.uint32), means=h(out.means), quats=h(out.quats),
                scales=h(out.scales))
    return res


def dump(name, res):
    """Save GPU results for offline analysis when TG_DUMP_DIR is set."""
    import os
    d = os.environ.get("TG_DUMP_DIR")
    if not d:
        return
    os.makedirs(d, exist_ok=True)
    np.savez_compressed(os.path.join(d, f"{name}.npz"),
                        **{k: v for k, v in res.items() if isinstance(v, np.ndarray)})


def compare_accumulators(acc, comp, rel=1e-4):
    """|gpu - oracle| <= rel * sum|term| + slack per entry (slack covers
    decisions within a band of their thresholds); counts within the number
    of marginal decisions.  Returns (n_bad, n_checked, info)."""
    mom, absm, slack, nmarg = comp["mom"], comp["absm"], comp["slack"], comp["nmarg"]
    a = acc[..., :15].astype(np.float64)
    m = mom[..., :15]
    tol = rel * absm[..., :15] + slack[..., :15] + 1e-30
    err = np.abs(a - m)
    bad = err > tol
    # counts (slots 12, 13) are integers: exact up to marginal decisions
    cnt_bad = np.abs(a[..., 12] - m[..., 12]) > nmarg
    bad[..., 12] = cnt_bad
    bad_rec = bad.any(-1)
    info = dict(worst=float((err / tol)[..., :12].max()) if err.size else 0.0,
                marginal_frac=float((slack[..., 0] > 0).mean()),
                bad_entries=int(bad.sum()))
    return int(bad_rec.sum()), int(bad_rec.size), info


def oracle_full(wl, raw=False):
    return oracle.motion_transfer(wl.scene, wl.cams, wl.disp, wl.vis, raw=raw)


def rotation_angle_deg(qa, qb):
    qa = qa / np.linalg.norm(qa, axis=-1, keepdims=True)
    qb = qb / np.linalg.norm(qb, axis=-1, keepdims=True)
    d = np.clip(np.abs((qa * qb).sum(-1)), 0, 1)
    return np.degrees(2 * np.arccos(d))


def sensitivity_mask(wl, ref, rel=1e-5, seeds=(1, 2), pos_tol=1e-3, rot_tol=0.05):
    """Gaussians whose oracle result moves by more than half the tolerance
    when the oracle's own FP64 accumulators are perturbed by `rel` (the size
    of FP32 accumulation error).  Those results are not determined at FP32
    input precision and are excluded from strict comparison."""
    comp, geom, cov = ref["comp"], ref["geom"], ref["cov"]
    unstable = np.zeros(wl.scene.n, bool)
    for s in seeds:
        rng = np.random.default_rng(s)
        mom = comp["mom"] * (1.0 + rel * rng.standard_normal(comp["mom"].shape))
        # decisions within a band of their thresholds may go the other way in
        # FP32: move each entry anywhere inside its slack bound, and the pixel
        # counts by up to the number of such decisions
        mom = mom + comp["slack"] * rng.uniform(-1.0, 1.0, comp["mom"].shape)
        mom[..., 12:] = comp["mom"][..., 12:]
        mom[..., 12] += np.round(comp["nmarg"] * rng.uniform(-1.0, 1.0, comp["nmarg"].shape))
        sv = oracle.solve_views(mom, geom.mu, cov, geom.valid)
        tri = oracle.triangulate(wl.scene, wl.cams, sv, mom, geom.valid)
        t0 = ref["tri"]
        unstable |= tri["status"] != t0["status"]
        unstable |= np.linalg.norm(tri["means"] - t0["means"], axis=-1) > 0.5 * pos_tol
        ang = rotation_angle_deg(tri["quats"], t0["quats"])
        unstable |= ang > 0.5 * rot_tol
        unstable |= np.abs(tri["scales"] / t0["scales"] - 1).max(-1) > 1e-3
        unstable |= (sv["flags"] != ref["sv"]["flags"]).any(0)
    return unstable


def eigen_gap(eig):
    e = np.sort(eig, axis=-1)
    return np.minimum(e[..., 1] - e[..., 0], e[..., 2] - e[..., 1]) / np.maximum(e[..., 2], 1e-300)


def check_end_to_end(case, wl, ref, gpu, max_unstable=0.05):
    """End-to-end parity of one frame (status, positions, rotations,
    scales, untouched copies) against the oracle; Gaussians whose oracle
    result is not determined at FP32 input precision are excluded, at most
    `max_unstable` of the updated ones (the fraction is logged)."""
    tri = ref["tri"]
    unstable = sensitivity_mask(wl, ref)
    st_g, st_o = gpu["status"], tri["status"]
    mism = (st_g != st_o) & ~unstable
    upd = (st_o & (oracle.ST_POS | oracle.ST_COV)) > 0
    frac = float(unstable.sum()) / max(1, int((upd | unstable).sum()))
    log(f"[{case}] status mismatches {mism.sum()} / {st_o.size}; unstable excluded {unstable.sum()} "
        f"({100 * frac:.2f}% of the {int((upd | unstable).sum())} updated or unstable Gaussians)")
    assert frac <= max_unstable, frac
    assert mism.sum() <= max(2, 2e-3 * st_o.size)
    pos = ((st_g & oracle.ST_POS) > 0) & ((st_o & oracle.ST_POS) > 0) & ~unstable
    dpos = np.linalg.norm(gpu["means"][pos].astype(np.float64) - tri["means"][pos], axis=-1)
    assert np.all(dpos <= 1e-3), dpos.max()
    cov = ((st_g & oracle.ST_COV) > 0) & ((st_o & oracle.ST_COV) > 0) & ~unstable
    gap = eigen_gap(tri["eig"])
    rot = cov & (gap >= 1e-2)
    ang = rotation_angle_deg(gpu["quats"][rot].astype(np.float64), tri["quats"][rot])
    assert np.all(ang <= 0.05), ang.max()
    assert np.all(gpu["quats"][rot][:, 0] >= 0)
    # degenerate eigen-gap: compare Sigma_3D' instead
    deg = cov & (gap < 1e-2)
    if deg.any():
        Rg = oracle.quat_to_rot(gpu["quats"][deg].astype(np.float64))
        Ro = oracle.quat_to_rot(tri["quats"][deg])
        Sg = Rg @ (gpu["scales"][deg][:, :, None] ** 2 * np.swapaxes(Rg, -1, -2))
        So = Ro @ (tri["scales"][deg][:, :, None] ** 2 * np.swapaxes(Ro, -1, -2))
        rel = np.linalg.norm(Sg - So, axis=(1, 2)) / np.linalg.norm(So, axis=(1, 2))
        assert np.all(rel <= 1e-3), rel.max()
    sc = np.abs(gpu["scales"][cov] / tri["scales"][cov] - 1)
    assert np.all(sc <= 1e-3), sc.max()
    # what was not updated is copied bit-exactly
    keep = (st_g & oracle.ST_POS) == 0
    np.testing.assert_array_equal(gpu["means"][keep], wl.scene.means[keep])
    keepc = (st_g & oracle.ST_COV) == 0
    np.testing.assert_array_equal(gpu["quats"][keepc], wl.scene.quats[keepc])
    np.testing.assert_array_equal(gpu["scales"][keepc], wl.scene.scales[keepc])
    log(f"[{case}] e2e: pos {pos.sum()} max {dpos.max() if dpos.size else 0:.2e}; rot {rot.sum()} "
        f"max {ang.max() if ang.size else 0:.2e} deg")


# ------------------------------------------------------------ stage checks
def check_preprocess(case, wl, ref, gpu):
    """a1: culling, depth keys, rectangles and centres bit-exact; FP64-formed
    conic and covariance within FP32 rounding."""
    g = ref["geom"]
    valid = g.valid.astype(bool)
    rect = gpu["rect"].astype(np.int32)
    gvalid = (rect[..., 2] > rect[..., 0]) & (rect[..., 3] > rect[..., 1])
    np.testing.assert_array_equal(gvalid, valid)
    # integer-deciding FP32 quantities: bit-exact
    np.testing.assert_array_equal(gpu["key"][valid], g.key[valid])
    np.testing.assert_array_equal(rect[valid], g.rect[valid])
    np.testing.assert_array_equal(gpu["rec"][..., 0:2][valid].view(np.uint32), g.mu[valid].view(np.uint32))
    # FP64-formed conic / covariance, rounded once to FP32
    conic = gpu["rec"][..., 2:5][valid].astype(np.float64)
    np.testing.assert_allclose(conic, ref["conic"][valid], rtol=2e-6, atol=1e-9 * np.abs(ref["conic"]).max())
    cov = gpu["cov2d"][valid].astype(np.float64)
    scale = np.abs(ref["cov"][valid]).max(-1, keepdims=True)
    assert np.all(np.abs(cov - ref["cov"][valid]) <= 2e-6 * scale + 1e-12)
    np.testing.assert_array_equal(gpu["rec"][..., 5][valid], np.broadcast_to(wl.scene.opacity, valid.shape)[valid])


def check_bins(case, wl, ref, gpu, expand=True):
    """a2: depth order, coarse lists and (with expand) the expanded per-tile
    lists bit-exact against the brute-force lists."""
    V, N = ref["geom"].key.shape
    assert gpu["overflow"] == 0
    orders = oracle.depth_order(ref["geom"])
    for v in range(V):
        o = orders[v]
        np.testing.assert_array_equal(gpu["order"][v, :o.size], o)
    mt = gpu["mt"]
    cell = 1 << 3
    starts, ids = oracle.cell_lists(ref["geom"], wl.cams, cell)
    assert gpu["n_pairs"] == ids.size
    rg = gpu["cell_ranges"].reshape(-1, 2)
    assert rg.shape[0] == starts.size - 1
    for c in range(rg.shape[0]):
        a, b = int(starts[c]), int(starts[c + 1])
        if a == b:
            assert rg[c, 0] == rg[c, 1]
            continue
        np.testing.assert_array_equal(gpu["cell_ids"][rg[c, 0]:rg[c, 1]], ids[a:b])
    if not expand:
        return
    # expanded per-tile lists equal the brute-force per-tile lists
    from paper_2604_02586_amd import api
    tids, tr = api.bin_expand(mt.splats, mt.bins, N, wl.cams, mt.params)
    tids = tids.cpu().numpy().view(np.uint32)
    tr = tr.cpu().numpy().view(np.uint32)
    ts, tl = oracle.cell_lists(ref["geom"], wl.cams, 1)
    assert tids.size == tl.size
    for t in range(tr.shape[0]):
        np.testing.assert_array_equal(tids[tr[t, 0]:tr[t, 1]], tl[ts[t]:ts[t + 1]])


def check_accumulate(case, wl, ref, gpu, max_marginal=0.02):
    """a3: every record within tolerance; T_final and pair counters when the
    launch recorded them."""
    comp = ref["comp"]
    nbad, ntot, info = compare_accumulators(gpu["acc"], comp)
    log(f"[{case}] accumulators: {nbad}/{ntot} outside tolerance, {info}")
    assert nbad == 0, info
    assert info["marginal_frac"] <= max_marginal, info
    if gpu["t_final"] is None:
        return
    # final transmittance per pixel (Sigma w = 1 - T_final), marginal pixels excluded
    ok = comp["pixmarg"] == 0
    np.testing.assert_allclose(gpu["t_final"][ok], comp["tfinal"][ok], rtol=1e-4, atol=1e-6)
    # pair counters in the sequential semantics: contributions are the same;
    # evaluations can only drop (exact culling of Gaussians whose alpha stays
    # below alpha_min on a whole tile)
    ev, ec = comp["counters"].sum(0)
    assert abs(int(gpu["stats"][1]) - ec) <= max(3, 1e-4 * ec)
    assert ec <= int(gpu["stats"][0]) <= ev + max(3, 1e-4 * ev)
    log(f"[{case}] pairs: evaluated {int(gpu['stats'][0])} (oracle lists {ev}), contributing "
        f"{int(gpu['stats'][1])}, pixel steps {int(gpu['stats'][2])}")


def check_solve(case, wl, ref, gpu):
    """a4: flags (away from thresholds), mu' and Sigma' on well-conditioned
    views."""
    sv = ref["sv"]
    comp = ref["comp"]
    # flags agree except where the oracle's value sits within 1e-3 of a threshold
    m = comp["mom"]
    near = (np.abs(m[..., oracle.S_W] / oracle.WSUM_MIN - 1) < 1e-3) | \
           (np.abs(sv["det"] / oracle.DET_MIN - 1) < 1e-2) | (comp["slack"][..., 0] > 0)
    diff = (gpu["vflags"] != sv["flags"]) & ~near
    assert diff.sum() <= max(2, 1e-3 * diff.size), (diff.sum(), diff.size)
    both = (gpu["vflags"] == oracle.VF_OK) & (sv["flags"] == oracle.VF_OK) & ~near
    # conditioning-aware: relative perturbation 1e-5 of the oracle's moments
    V1, _ = oracle.v1_v2(m[both])
    cond = np.full(both.shape, np.inf)
    cond[both] = np.linalg.cond(V1)
    well = both & (cond < 1e4)
    err_mu = np.abs(gpu["mu_new"][well] - sv["mu_new"][well]).max(-1)
    assert np.all(err_mu <= 1e-2 + 1e-6 * cond[well] * 10), err_mu.max()
    # Eq. 2: Sigma_2D' = A Sigma_2D A^T, relative to its largest entry
    cg, co = gpu["cov_new"][well].astype(np.float64), sv["cov_new"][well]
    err_cov = np.abs(cg - co).max(-1) / np.abs(co).max(-1)
    assert np.all(err_cov <= 2e-3 + 1e-6 * cond[well] * 10), err_cov.max()
    log(f"[{case}] solve: {well.sum()} well-conditioned views, max |dmu'| = {err_mu.max():.2e} px, "
        f"max rel dSigma' = {err_cov.max():.2e}")


