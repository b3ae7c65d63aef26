"""Invariants and exact recovery through libtg (Sec. 4.3.4 Eq. 4, Sec. 4.4),
and the non-finite input rules.

- Identity tracks (d = 0): the per-view solve gives A = I and c = 0 exactly
  (every displacement sum is exactly zero), so mu' and Sigma' are the
  splat's own centre and covariance bit for bit, and the update returns the
  Gaussian where it was.
- A constant shift delta_v per view: A = I and c = delta_v for every solved
  (Gaussian, view), within the FP32 accumulation.
- Single Gaussians moved rigidly, with tracks from the Gaussian optimal-
  transport (Monge) map between the projected covariances before and after
  (V = 3..8 views): the update recovers the known mean, rotation and scales.
- Non-finite inputs: a Gaussian with a non-finite parameter and the views a
  non-finite track reaches are flagged exactly as the oracle flags them.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from helpers import check_end_to_end, log, oracle_full, rotation_angle_deg, run_gpu

pytestmark = pytest.mark.gpu


def _lite(seed=5, n=20000):
    return synth.make_workload("medium", seed=seed, n=n, views=5, width=420, height=300)


def _with_disp(wl, disp, vis=None):
    return synth.Workload(name=wl.name, scene=wl.scene, cams=wl.cams, motion=wl.motion,
                          disp=np.ascontiguousarray(disp, np.float32),
                          vis=np.ones_like(wl.vis) if vis is None else vis)


def test_identity_tracks_leave_everything_in_place():
    wl = _with_disp(_lite(), np.zeros_like(_lite().disp))
    gpu = run_gpu(wl)
    ok = gpu["vflags"] == oracle.VF_OK
    assert ok.mean() > 0.2
    # Theta = V1^-1 * 0 exactly: the new 2D mean and covariance are the old ones
    np.testing.assert_array_equal(gpu["mu_new"][ok].view(np.uint32), gpu["rec"][..., 0:2][ok].view(np.uint32))
    np.testing.assert_array_equal(gpu["cov_new"][ok].view(np.uint32), gpu["cov2d"][ok].view(np.uint32))
    st = gpu["status"]
    pos = (st & oracle.ST_POS) > 0
    assert pos.mean() > 0.2
    d = np.linalg.norm(gpu["means"][pos].astype(np.float64) - wl.scene.means[pos], axis=-1)
    log(f"identity: {pos.sum()} positions, max |mu' - mu| = {d.max():.2e}")
    assert d.max() <= 1e-4
    ref = oracle_full(wl)
    check_end_to_end("identity", wl, ref, gpu)
    cov = ((st & oracle.ST_COV) > 0) & (ref["tri"]["status"] & oracle.ST_COV > 0)
    sc = np.abs(gpu["scales"][cov] / wl.scene.scales[cov] - 1)
    log(f"identity: {cov.sum()} covariances, median |s'/s - 1| = {np.median(sc):.2e}")
    assert np.median(sc) <= 1e-4


def test_constant_shift_per_view():
    base = _lite(seed=6)
    V = len(base.cams)
    shift = np.array([[1.5, -0.5], [0.0, 2.0], [-1.0, -1.0], [0.7, 0.3], [-2.5, 1.25]])[:V]
    disp = np.broadcast_to(shift[:, None, None, :], base.disp.shape)
    wl = _with_disp(base, disp)
    gpu = run_gpu(wl)
    ref = oracle_full(wl)
    ok = (gpu["vflags"] == oracle.VF_OK) & (ref["sv"]["flags"] == oracle.VF_OK)
    V1, _ = oracle.v1_v2(ref["comp"]["mom"][ok])
    cond = np.linalg.cond(V1)
    well = cond < 1e4
    c = gpu["mu_new"][ok].astype(np.float64) - gpu["rec"][..., 0:2][ok]
    dc = np.abs(c - np.broadcast_to(shift[:, None, :], ok.shape + (2,))[ok]).max(-1)
    log(f"shift: {ok.sum()} solved views ({well.sum()} well conditioned), max |c - delta| = {dc[well].max():.2e} px")
    assert dc[well].max() <= 1e-3
    cg, c0 = gpu["cov_new"][ok][well].astype(np.float64), gpu["cov2d"][ok][well].astype(np.float64)
    rel = np.abs(cg - c0).max(-1) / np.abs(c0).max(-1)
    assert rel.max() <= 1e-3, rel.max()
    check_end_to_end("shift", wl, ref, gpu)


def _monge(S, Sp):
    def sqrtm(M):
        w, U = np.linalg.eigh(M)
        return U @ np.diag(np.sqrt(w)) @ U.T
    Sh = sqrtm(S)
    Shi = np.linalg.inv(Sh)
    return Shi @ sqrtm(Sh @ Sp @ Sh) @ Shi


@pytest.mark.parametrize("V", [3, 4, 6, 8])
def test_exact_recovery_of_rigid_motion(V):
    """Known rigid motions of single Gaussians (rotation up to 30 degrees,
    translation up to 0.3) recovered through the whole GPU path from FP32
    tracks of the Monge map."""
    rng = np.random.default_rng(200 + V)
    cams = synth.hemisphere_cameras(V, 3.0, 160, 160, fov_x_deg=50.0)
    worst = [0.0, 0.0, 0.0]
    for trial in range(8):
        mu = rng.uniform(-0.15, 0.15, 3)
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        q[0] = abs(q[0])
        s = np.sort(rng.uniform(0.06, 0.12, 3))[rng.permutation(3)]
        rot = Rotation.from_rotvec(rng.standard_normal(3) / math.sqrt(3) * math.radians(rng.uniform(0, 30)))
        t = rng.standard_normal(3)
        t *= rng.uniform(0, 0.3) / np.linalg.norm(t)
        R_n = rot.as_matrix() @ Rotation.from_quat([*q[1:], q[0]]).as_matrix()
        qn = Rotation.from_matrix(R_n).as_quat()[[3, 0, 1, 2]]
        qn *= np.sign(qn[0])
        mk = lambda m, qq: synth.Scene(means=np.asarray([m], np.float32), quats=np.asarray([qq], np.float32),
                                       scales=np.asarray([s], np.float32), opacity=np.array([0.9], np.float32),
                                       rgb=np.zeros((1, 3), np.float32))
        sc, moved = mk(mu, q), mk(mu + t, qn)
        g = oracle.geometry(sc, cams)
        cov0, _ = oracle.project64(sc, cams)
        cov1, _ = oracle.project64(moved, cams)
        disp = np.zeros((V, 160, 160, 2))
        cc, rr = np.meshgrid(np.arange(160.0), np.arange(160.0))
        for v, cam in enumerate(cams):
            S0 = np.array([[cov0[v, 0, 0], cov0[v, 0, 1]], [cov0[v, 0, 1], cov0[v, 0, 2]]])
            S1 = np.array([[cov1[v, 0, 0], cov1[v, 0, 1]], [cov1[v, 0, 1], cov1[v, 0, 2]]])
            A = _monge(S0, S1)
            p = cam.R.astype(np.float64) @ moved.means[0].astype(np.float64) + cam.t.astype(np.float64)
            x1 = np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])
            b = x1 - A @ g.mu[v, 0].astype(np.float64)
            disp[v, ..., 0] = A[0, 0] * cc + A[0, 1] * rr + b[0] - cc
            disp[v, ..., 1] = A[1, 0] * cc + A[1, 1] * rr + b[1] - rr
        wl = synth.Workload(name="monge", scene=sc, cams=cams, motion=None, disp=disp.astype(np.float32),
                            vis=np.ones((V, 160, 160), np.uint8))
        gpu = run_gpu(wl)
        assert gpu["status"][0] == oracle.ST_POS | oracle.ST_COV, (trial, gpu["status"][0], gpu["vflags"][:, 0])
        dpos = float(np.linalg.norm(gpu["means"][0].astype(np.float64) - moved.means[0]))
        ang = float(rotation_angle_deg(gpu["quats"][0:1].astype(np.float64), moved.quats[0:1].astype(np.float64))[0])
        dsc = float(np.abs(gpu["scales"][0] / s - 1).max())
        worst = [max(worst[0], dpos), max(worst[1], ang), max(worst[2], dsc)]
        assert dpos <= 1e-3 and ang <= 0.05 and dsc <= 1e-3, (trial, dpos, ang, dsc)
    log(f"V={V}: worst position {worst[0]:.2e}, rotation {worst[1]:.2e} deg, scale {worst[2]:.2e}")


def test_nonfinite_inputs_are_flagged_like_the_oracle():
    base = _lite(seed=8, n=12000)
    rng = np.random.default_rng(3)
    sc = synth.Scene(means=base.scene.means.copy(), quats=base.scene.quats.copy(), scales=base.scene.scales.copy(),
                     opacity=base.scene.opacity.copy(), rgb=base.scene.rgb)
    bad = rng.choice(sc.n, 60, replace=False)
    for k, i in enumerate(bad):
        [sc.means, sc.quats, sc.scales][k % 3][i, k % 3] = [np.nan, np.inf, -np.inf][k % 3]
    sc.opacity[bad[::7]] = np.nan
    disp = base.disp.copy()
    V, H, W = base.vis.shape
    pv, py, px = rng.integers(0, V, 40), rng.integers(0, H, 40), rng.integers(0, W, 40)
    disp[pv, py, px, rng.integers(0, 2, 40)] = np.nan
    wl = synth.Workload(name=base.name, scene=sc, cams=base.cams, motion=None, disp=disp, vis=base.vis)
    gpu = run_gpu(wl)
    ref = oracle_full(wl)
    st_g, st_o = gpu["status"], ref["tri"]["status"]
    nf_g, nf_o = (st_g & oracle.ST_NONFINITE) > 0, (st_o & oracle.ST_NONFINITE) > 0
    log(f"non-finite: {nf_o.sum()} flagged by the oracle, {nf_g.sum()} by the GPU; "
        f"views with flag 32: {int(((ref['sv']['flags'] & 32) > 0).sum())}")
    np.testing.assert_array_equal(nf_g, nf_o)
    assert nf_g[bad].all()
    np.testing.assert_array_equal((gpu["vflags"] & 32) > 0, (ref["sv"]["flags"] & 32) > 0)
    np.testing.assert_array_equal(gpu["vflags"][:, bad], oracle.VF_CULLED | oracle.VF_FEW_PIX | oracle.VF_LOW_ALPHA
                                  | oracle.VF_SINGULAR)
    assert not (st_g[bad] & (oracle.ST_POS | oracle.ST_COV)).any()
    fin = np.ones(sc.n, bool)
    fin[bad] = False
    assert np.isfinite(gpu["means"][fin]).all() and np.isfinite(gpu["quats"][fin]).all()
    check_end_to_end("nonfinite", wl, ref, gpu)
