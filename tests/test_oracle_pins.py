"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, finite differences, textbook library routines (scipy rotations,
numpy least squares), brute force on tiny inputs, invariants, and exact
recovery of a known rigid motion.  None needs a GPU.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ----------------------------------------------------------------- helpers
def scene_of(means, quats, scales, opacity):
    means = np.atleast_2d(np.asarray(means, np.float32))
    n = means.shape[0]
    return synth.Scene(means=means, quats=np.atleast_2d(np.asarray(quats, np.float32)),
                       scales=np.atleast_2d(np.asarray(scales, np.float32)),
                       opacity=np.asarray(opacity, np.float32).reshape(n),
                       rgb=np.zeros((n, 3), np.float32))


def axis_camera(z0, W=64, H=64, f=80.0):
    """Camera at (0,0,-z0) looking along +z (R = I, t = (0,0,z0))."""
    return synth.Camera(R=np.eye(3, dtype=np.float32), t=np.array([0, 0, z0], np.float32), fx=f, fy=f,
                        cx=(W - 1) / 2, cy=(H - 1) / 2, W=W, H=H)


def pinhole(cam, X):
    p = np.asarray(X, np.float64) @ cam.R.astype(np.float64).T + cam.t.astype(np.float64)
    return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy]), p


def sigma3(q_wxyz, s):
    R = Rotation.from_quat([q_wxyz[1], q_wxyz[2], q_wxyz[3], q_wxyz[0]]).as_matrix()
    return R @ np.diag(np.asarray(s, np.float64) ** 2) @ R.T


# ----------------------------------------------------------------- P1: projection (Eq. 1)
def test_p1_axis_aligned_closed_form():
    z0, sx, sy, sz = 4.0, 0.05, 0.02, 0.03
    cam = axis_camera(z0)
    sc = scene_of([[0, 0, 0]], [[1, 0, 0, 0]], [[sx, sy, sz]], [0.5])
    cov, conic = oracle.project64(sc, [cam])
    f = np.float64(np.float32(80.0))
    np.testing.assert_allclose(cov[0, 0], [f * f * sx * sx / z0 ** 2, 0.0, f * f * sy * sy / z0 ** 2],
                               rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(conic[0, 0], [1 / (cov[0, 0, 0] + 0.3), 0.0, 1 / (cov[0, 0, 2] + 0.3)], rtol=1e-12)


def test_p1_jacobian_by_finite_differences():
    rng = np.random.default_rng(7)
    cams = synth.ring_cameras(3, 3.0, 128, 96)
    for _ in range(20):
        mu = rng.uniform(-0.3, 0.3, 3)
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        s = rng.uniform(0.02, 0.08, 3)
        sc = scene_of([mu], [q], [s], [0.5])
        cov, _ = oracle.project64(sc, cams)
        S3 = sigma3(sc.quats[0].astype(np.float64), sc.scales[0].astype(np.float64))
        for v, cam in enumerate(cams):
            _, p = pinhole(cam, sc.means[0])
            J = np.zeros((2, 3))
            h = 1e-6
            for k in range(3):
                e = np.zeros(3)
                e[k] = h
                f = lambda pp: np.array([cam.fx * pp[0] / pp[2], cam.fy * pp[1] / pp[2]])
                J[:, k] = (f(p + e) - f(p - e)) / (2 * h)
            W = cam.R.astype(np.float64)
            ref = J @ W @ S3 @ W.T @ J.T
            np.testing.assert_allclose(cov[v, 0], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-6,
                                       atol=1e-8 * np.abs(ref).max())


def test_p1_rotation_about_optical_axis_rotates_sigma2d():
    cam = axis_camera(5.0)
    s = [0.08, 0.02, 0.03]
    base = scene_of([[0, 0, 0]], [[1, 0, 0, 0]], [s], [0.5])
    c0, _ = oracle.project64(base, [cam])
    S0 = np.array([[c0[0, 0, 0], c0[0, 0, 1]], [c0[0, 0, 1], c0[0, 0, 2]]])
    for th in (0.3, 1.0, 2.5):
        q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
        c1, _ = oracle.project64(scene_of([[0, 0, 0]], [q], [s], [0.5]), [cam])
        Rz = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        ref = Rz @ S0 @ Rz.T
        np.testing.assert_allclose(c1[0, 0], [ref[0, 0], ref[0, 1], ref[1, 1]], rtol=1e-6, atol=1e-9)


def test_p1_fp32_geometry_decisions():
    wl = synth.make_workload("small", seed=11, with_tracks=False)
    g = oracle.geometry(wl.scene, wl.cams)
    cov, _ = oracle.project64(wl.scene, wl.cams)
    for v, cam in enumerate(wl.cams):
        for i in range(0, wl.scene.n, 37):
            x, p = pinhole(cam, wl.scene.means[i])
            if p[2] <= 0.2:
                assert g.valid[v, i] == 0 and g.key[v, i] == 0xFFFFFFFF
                continue
            assert g.key[v, i] == np.float32(p[2]).view(np.uint32) or \
                abs(np.uint32(g.key[v, i]).view(np.float32) - p[2]) < 1e-6 * p[2]
            if not g.valid[v, i]:
                continue
            np.testing.assert_allclose(g.mu[v, i], x, atol=2e-4)
            Sr = np.array([[cov[v, i, 0] + 0.3, cov[v, i, 1]], [cov[v, i, 1], cov[v, i, 2] + 0.3]])
            r = 3.0 * math.sqrt(np.linalg.eigvalsh(Sr).max())
            TX, TY = -(-cam.W // 16), -(-cam.H // 16)
            x0, y0, x1, y1 = g.rect[v, i]
            # rectangle covers the 3-sigma square (clipped to the image tiles)
            assert x0 <= max(0, math.floor((x[0] - r) / 16)) and x1 >= min(TX, math.floor((x[0] + r) / 16) + 1)
            assert y0 <= max(0, math.floor((x[1] - r) / 16)) and y1 >= min(TY, math.floor((x[1] + r) / 16) + 1)


# ----------------------------------------------------------------- P2/P3: compositing
def _single_pixel_run(sc, cam, px, py, disp=(0.0, 0.0), vis=1):
    g = oracle.geometry(sc, [cam])
    cov, conic = oracle.project64(sc, [cam])
    lists = oracle.cell_lists(g, [cam], 1)
    d = np.zeros((1, cam.H, cam.W, 2), np.float32)
    d[0, py, px] = disp
    vv = np.zeros((1, cam.H, cam.W), np.uint8)
    vv[0, py, px] = vis
    pm = np.zeros((1, cam.H, cam.W), np.uint8)
    pm[0, py, px] = 1
    return g, cov, conic, oracle.composite(sc, [cam], g, conic, lists, d, vv, pixmask=pm, raw=True)


def test_p2_single_gaussian_single_pixel_closed_form():
    cam = axis_camera(4.0, W=64, H=64)
    s = [0.1, 0.06, 0.05]
    sc = scene_of([[0, 0, 0]], [[1, 0, 0, 0]], [s], [0.7])
    px, py = 36, 30
    g, cov, conic, r = _single_pixel_run(sc, cam, px, py, disp=(2.5, -1.0))
    f = np.float64(np.float32(80.0))
    s32 = np.asarray(s, np.float32).astype(np.float64)
    a = f * f * s32[0] ** 2 / 16 + 0.3
    c = f * f * s32[1] ** 2 / 16 + 0.3
    mu = g.mu[0, 0].astype(np.float64)
    ux, uy = px - mu[0], py - mu[1]
    alpha = min(0.99, float(np.float32(0.7)) * math.exp(-0.5 * (ux * ux / a + uy * uy / c)))
    m = r["mom"][0, 0]
    np.testing.assert_allclose(m[oracle.S_W], alpha, rtol=1e-9)
    np.testing.assert_allclose(m[oracle.S_UX], alpha * ux, rtol=1e-5)
    np.testing.assert_allclose(m[oracle.S_UXUY], alpha * ux * uy, rtol=1e-5)
    np.testing.assert_allclose(m[oracle.S_UYDX], alpha * uy * 2.5, rtol=1e-5)
    np.testing.assert_allclose(m[oracle.S_DY], -alpha, rtol=1e-5)
    assert m[oracle.S_N] == 1.0 and m[oracle.S_STATN] == 0.0
    np.testing.assert_allclose(r["tfinal"][0, py, px], 1 - alpha, rtol=1e-12)


def test_p2_two_gaussians_front_to_back():
    cam = axis_camera(4.0)
    sc = scene_of([[0, 0, 0.5], [0, 0, -0.5]], [[1, 0, 0, 0]] * 2, [[0.1, 0.1, 0.1], [0.12, 0.12, 0.12]], [0.6, 0.8])
    px = py = 31
    g, cov, conic, r = _single_pixel_run(sc, cam, px, py)
    # the second Gaussian (z = -0.5) is nearer the camera at z = -4
    al = []
    for i in range(2):
        mu = g.mu[0, i].astype(np.float64)
        d = np.array([px - mu[0], py - mu[1]])
        cn = conic[0, i]
        power = -0.5 * (cn[0] * d[0] ** 2 + cn[2] * d[1] ** 2) - cn[1] * d[0] * d[1]
        al.append(min(0.99, float(sc.opacity[i]) * math.exp(power)))
    w = r["mom"][0, :, oracle.S_W]
    np.testing.assert_allclose(w[1], al[1], rtol=1e-12)
    np.testing.assert_allclose(w[0], al[0] * (1 - al[1]), rtol=1e-12)


def test_p2_termination_stack():
    cam = axis_camera(4.0, W=63, H=63)
    k = 6
    sc = scene_of([[0, 0, 0.1 * i] for i in range(k)], [[1, 0, 0, 0]] * k, [[0.1, 0.1, 0.1]] * k, [0.95] * k)
    px = py = 31  # exactly the centre: alpha = 0.95, T = 1, 0.05, 0.0025, 1.25e-4
    g, cov, conic, r = _single_pixel_run(sc, cam, px, py)
    w = r["mom"][0, :, oracle.S_W]
    n = r["mom"][0, :, oracle.S_N]
    assert int(n.sum()) == 3, n                       # T: 1, ~0.05, ~0.0025, stop before < 1e-4
    assert np.all(n[:3] == 1) and np.all(n[3:] == 0)   # nearest (index 0) first
    np.testing.assert_allclose(w.sum(), 1 - r["tfinal"][0, py, px], rtol=1e-12)
    np.testing.assert_allclose(r["tfinal"][0, py, px], 0.05 ** 3, rtol=1e-6)


def test_p3_weights_sum_to_one_minus_final_transmittance():
    wl = synth.make_workload("small", seed=5)
    vis = np.ones_like(wl.vis)
    g = oracle.geometry(wl.scene, wl.cams)
    cov, conic = oracle.project64(wl.scene, wl.cams)
    lists = oracle.cell_lists(g, wl.cams, 1)
    r = oracle.composite(wl.scene, wl.cams, g, conic, lists, wl.disp, vis)
    lhs = r["mom"][..., oracle.S_W].sum(1)
    rhs = (1.0 - r["tfinal"]).reshape(len(wl.cams), -1).sum(1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10)
    assert np.all(r["tfinal"] <= 1.0) and np.all(r["tfinal"] >= 0.0)
    # counters: every contribution was evaluated
    assert np.all(r["counters"][:, 1] <= r["counters"][:, 0])


# ----------------------------------------------------------------- P4: binning by brute force
@pytest.mark.parametrize("cell", [1, 2, 8])
def test_p4_tile_lists_brute_force(cell):
    wl = synth.make_workload("small", seed=3, n=400, with_tracks=False)
    g = oracle.geometry(wl.scene, wl.cams)
    starts, ids = oracle.cell_lists(g, wl.cams, cell)
    base = 0
    for v, cam in enumerate(wl.cams):
        TX, TY = -(-cam.W // 16), -(-cam.H // 16)
        CX, CY = -(-TX // cell), -(-TY // cell)
        for cy in range(CY):
            for cx in range(CX):
                # brute force: Gaussians whose tile rectangle meets cell (cx, cy)
                sel = []
                for i in range(wl.scene.n):
                    if not g.valid[v, i]:
                        continue
                    x0, y0, x1, y1 = g.rect[v, i]
                    if x0 < (cx + 1) * cell and x1 > cx * cell and y0 < (cy + 1) * cell and y1 > cy * cell:
                        sel.append(i)
                sel = np.array(sel, np.int64)
                order = sel[np.lexsort((sel, g.key[v, sel].astype(np.int64)))] if sel.size else sel
                c = base + cy * CX + cx
                np.testing.assert_array_equal(ids[starts[c]:starts[c + 1]], order)
        base += CX * CY


def test_p4_filtered_coarse_lists_equal_tile_lists():
    """The coarse-bin design: filtering a coarse bin's depth-ordered list by
    the tile rectangle gives exactly the tile's depth-ordered list."""
    wl = synth.make_workload("small", seed=9, n=1500, with_tracks=False)
    g = oracle.geometry(wl.scene, wl.cams)
    ts, tids = oracle.cell_lists(g, wl.cams, 1)
    for cell in (2, 4, 8):
        cs, cids = oracle.cell_lists(g, wl.cams, cell)
        tb = cb = 0
        for v, cam in enumerate(wl.cams):
            TX, TY = -(-cam.W // 16), -(-cam.H // 16)
            CX = -(-TX // cell)
            for ty in range(TY):
                for tx in range(TX):
                    c = cb + (ty // cell) * CX + tx // cell
                    lst = cids[cs[c]:cs[c + 1]]
                    r = g.rect[v, lst]
                    keep = lst[(r[:, 0] <= tx) & (r[:, 2] > tx) & (r[:, 1] <= ty) & (r[:, 3] > ty)]
                    t = tb + ty * TX + tx
                    np.testing.assert_array_equal(keep, tids[ts[t]:ts[t + 1]])
            tb += TX * TY
            cb += CX * (-(-TY // cell))


# ----------------------------------------------------------------- P5/P6: LS (Eq. 3 = Eq. 4)
def _single_gaussian_frame(seed, disp_fn, W=96, H=96, s=(0.12, 0.07, 0.09)):
    rng = np.random.default_rng(seed)
    cam = axis_camera(4.0, W, H, f=100.0)
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    sc = scene_of([rng.uniform(-0.1, 0.1, 3)], [q], [s], [0.8])
    cc, rr = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    d = disp_fn(cc, rr).astype(np.float32)[None]
    return sc, cam, d


def test_p5_incremental_equals_naive_weighted_lstsq():
    rng = np.random.default_rng(1)
    noise = rng.normal(0, 0.7, (96, 96, 2))
    fn = lambda c, r: np.stack([0.05 * c - 0.02 * r + 1.5, 0.01 * c + 0.03 * r - 2.0], -1) + noise
    sc, cam, d = _single_gaussian_frame(2, fn)
    r = oracle.motion_transfer(sc, [cam], d, np.ones((1, 96, 96), np.uint8), raw=True)
    g, conic = r["geom"], r["conic"]
    # naive weighted least squares over the explicitly stacked pixels (Eq. 3)
    mu = g.mu[0, 0].astype(np.float64)
    x0, y0, x1, y1 = g.rect[0, 0]
    rows, rhs, wts = [], [], []
    for py in range(y0 * 16, min(96, y1 * 16)):
        for px in range(x0 * 16, min(96, x1 * 16)):
            dd = np.array([px - mu[0], py - mu[1]])
            cn = conic[0, 0]
            power = -0.5 * (cn[0] * dd[0] ** 2 + cn[2] * dd[1] ** 2) - cn[1] * dd[0] * dd[1]
            a = min(0.99, float(np.float32(0.8)) * math.exp(power))
            if a < 1 / 255:
                continue
            rows.append([px, py, 1.0])
            rhs.append([px + float(d[0, py, px, 0]), py + float(d[0, py, px, 1])])
            wts.append(a)
    X, Y, w = np.array(rows), np.array(rhs, np.float64), np.array(wts)
    sol, *_ = np.linalg.lstsq(X * np.sqrt(w)[:, None], Y * np.sqrt(w)[:, None], rcond=None)
    A_ref, b_ref = sol[:2].T, sol[2]
    sv = r["sv"]
    assert sv["flags"][0, 0] == oracle.VF_OK
    A = sv["A"][0, 0]
    b = sv["mu_new"][0, 0] - A @ mu
    np.testing.assert_allclose(A, A_ref, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(b, b_ref, rtol=1e-9, atol=1e-8)
    # paper-literal raw-coordinate V1, V2 (Eq. 4) give the same solution
    raw = r["comp"]["raw"][0, 0]
    V1 = raw[:9].reshape(3, 3)
    V2 = raw[9:].reshape(3, 2)
    th = np.linalg.solve(V1, V2)
    np.testing.assert_allclose(th[:2].T, A_ref, rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(th[2], b_ref, rtol=1e-7, atol=1e-6)


def test_p5_raw_and_centred_agree_on_overlapping_scene():
    wl = synth.make_workload("small", seed=4, n=600)
    r = oracle.motion_transfer(wl.scene, wl.cams, wl.disp, wl.vis, raw=True)
    sv = r["sv"]
    raw = r["comp"]["raw"]
    ok = sv["flags"] == oracle.VF_OK
    V1 = raw[..., :9].reshape(raw.shape[:2] + (3, 3))[ok]
    V2 = raw[..., 9:].reshape(raw.shape[:2] + (3, 2))[ok]
    cond = np.linalg.cond(V1)
    good = cond < 1e8
    th = np.linalg.solve(V1[good], V2[good])
    A_raw = np.swapaxes(th[:, :2], -1, -2)
    mu = r["geom"].mu.astype(np.float64)[ok][good]
    mu_raw = np.einsum("nij,nj->ni", A_raw, mu) + th[:, 2]
    np.testing.assert_allclose(A_raw, sv["A"][ok][good], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(mu_raw, sv["mu_new"][ok][good], rtol=1e-8, atol=1e-5)


def test_p6_exact_affine_tracks_recovered():
    A_true = np.array([[1.08, -0.05], [0.03, 0.95]])
    b_true = np.array([3.0, -1.5])
    fn = lambda c, r: np.stack([A_true[0, 0] * c + A_true[0, 1] * r + b_true[0] - c,
                                A_true[1, 0] * c + A_true[1, 1] * r + b_true[1] - r], -1)
    sc, cam, d = _single_gaussian_frame(3, fn)
    # FP32 tracks: compare against the affine map the FP32 field encodes
    r = oracle.motion_transfer(sc, [cam], d.astype(np.float64), np.ones((1, 96, 96), np.uint8))
    sv = r["sv"]
    mu = r["geom"].mu[0, 0].astype(np.float64)
    A = sv["A"][0, 0]
    b = sv["mu_new"][0, 0] - A @ mu
    np.testing.assert_allclose(A, A_true, atol=2e-7)
    np.testing.assert_allclose(b, b_true, atol=5e-5)
    np.testing.assert_allclose(sv["cov_new"][0, 0], (A @ np.array([[r["cov"][0, 0, 0], r["cov"][0, 0, 1]],
                                                                  [r["cov"][0, 0, 1], r["cov"][0, 0, 2]]]) @ A.T)
                               [[0, 0, 1], [0, 1, 1]], rtol=1e-12)


# ----------------------------------------------------------------- P7-P9: multi-view update
def _fake_sv(cams, mu3, Sigma3):
    """Exact per-view 2D means and covariances of a 3D Gaussian."""
    V = len(cams)
    mu_new = np.zeros((V, 1, 2))
    rows, _ = oracle.cov_rows(cams, mu3[None])
    sig6 = np.array([Sigma3[0, 0], Sigma3[0, 1], Sigma3[0, 2], Sigma3[1, 1], Sigma3[1, 2], Sigma3[2, 2]])
    cov_new = np.einsum("vnij,j->vni", rows, sig6)
    for v, cam in enumerate(cams):
        mu_new[v, 0], _ = pinhole(cam, mu3)
    flags = np.full((V, 1), oracle.VF_OK, np.uint8)
    mom = np.zeros((V, 1, 16))
    mom[..., oracle.S_W] = 1.0
    mom[..., oracle.S_N] = 10
    return dict(flags=flags, mu_new=mu_new, cov_new=cov_new), mom


@pytest.mark.parametrize("V", [2, 3, 5, 8])
def test_p7_p8_p9_exact_triangulation_and_covariance(V):
    rng = np.random.default_rng(V)
    cams = synth.hemisphere_cameras(V, 4.0, 200, 160)
    for _ in range(5):
        mu3 = rng.uniform(-0.4, 0.4, 3)
        q_old = rng.standard_normal(4)
        q_old /= np.linalg.norm(q_old)
        s_old = np.sort(rng.uniform(0.02, 0.08, 3))[rng.permutation(3)]
        rot = Rotation.from_rotvec(rng.standard_normal(3) * 0.3)
        R_new = rot.as_matrix() @ Rotation.from_quat([*q_old[1:], q_old[0]]).as_matrix()
        s_new = s_old * rng.uniform(0.9, 1.1, 3)
        Sig = R_new @ np.diag(s_new ** 2) @ R_new.T
        sv, mom = _fake_sv(cams, mu3, Sig)
        sc = scene_of([[0, 0, 0]], [q_old], [s_old], [0.5])
        tri = oracle.triangulate(sc, cams, sv, mom, np.ones((V, 1), np.uint8))
        np.testing.assert_allclose(tri["means"][0], mu3, atol=1e-10)
        if V == 2:
            # Two views constrain only 5 of the 6 covariance unknowns: the
            # symmetric matrix r1 r2^T + r2 r1^T of the two viewing rays is in
            # the kernel of both views' maps.  The update is rejected.
            assert tri["status"][0] == oracle.ST_POS | oracle.ST_NEG_EIG
            rows, _ = oracle.cov_rows(cams, mu3[None])
            A = rows[:, 0].reshape(6, 6)
            assert np.linalg.matrix_rank(A, tol=1e-9 * np.abs(A).max()) == 5
            continue
        assert tri["status"][0] == oracle.ST_POS | oracle.ST_COV
        Rq = Rotation.from_quat([*tri["quats"][0][1:], tri["quats"][0][0]]).as_matrix()
        s = tri["scales"][0]
        np.testing.assert_allclose(Rq @ np.diag(s ** 2) @ Rq.T, Sig, rtol=1e-8, atol=1e-12)
        if np.all(np.argsort(s_new) == np.argsort(s_old.astype(np.float32))):
            np.testing.assert_allclose(Rq, R_new, atol=1e-7)
            np.testing.assert_allclose(s, s_new, rtol=1e-8)
        assert tri["quats"][0][0] >= 0


def test_p9_quaternion_round_trip_and_shepperd():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((500, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1
    R = oracle.quat_to_rot(q)
    R_ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(R, R_ref, atol=1e-12)
    np.testing.assert_allclose(oracle.rot_to_quat(R), q, atol=1e-12)
    # near-180-degree rotations exercise the non-trace pivots
    q2 = np.array([[1e-9, 1, 0, 0], [1e-9, 0, 1, 0], [1e-9, 0, 0, 1], [0.01, 0.7, 0.7, 0.1]])
    q2 /= np.linalg.norm(q2, axis=1, keepdims=True)
    np.testing.assert_allclose(oracle.quat_to_rot(oracle.rot_to_quat(oracle.quat_to_rot(q2))),
                               oracle.quat_to_rot(q2), atol=1e-12)


def test_p9_reorder_keeps_first_frame_axis_order():
    """Eigenvalues come out sorted; the update must keep each axis with its
    own scale (Sec. 4.4.3): an unrotated Gaussian with scales (3,1,2) stays
    (3,1,2) with the identity rotation."""
    cams = synth.hemisphere_cameras(4, 4.0, 200, 160)
    s_old = np.array([0.06, 0.02, 0.04])
    Sig = np.diag(s_old ** 2 * 1.1)
    sv, mom = _fake_sv(cams, np.zeros(3), Sig)
    sc = scene_of([[0, 0, 0]], [[1, 0, 0, 0]], [s_old], [0.5])
    tri = oracle.triangulate(sc, cams, sv, mom, np.ones((4, 1), np.uint8))
    np.testing.assert_allclose(tri["scales"][0], s_old * math.sqrt(1.1), rtol=1e-9)
    np.testing.assert_allclose(tri["quats"][0], [1, 0, 0, 0], atol=1e-9)


def test_p9_negative_eigenvalue_keeps_old_rotation_and_scale():
    cams = synth.hemisphere_cameras(3, 4.0, 200, 160)
    Sig = np.diag([1e-3, 4e-4, -1e-4])
    sv, mom = _fake_sv(cams, np.array([0.1, 0.0, 0.0]), Sig)
    q_old = np.array([0.9, 0.1, 0.2, 0.3]) / np.linalg.norm([0.9, 0.1, 0.2, 0.3])
    sc = scene_of([[0, 0, 0]], [q_old], [[0.03, 0.02, 0.01]], [0.5])
    tri = oracle.triangulate(sc, cams, sv, mom, np.ones((3, 1), np.uint8))
    assert tri["status"][0] == oracle.ST_POS | oracle.ST_NEG_EIG
    np.testing.assert_allclose(tri["means"][0], [0.1, 0, 0], atol=1e-10)
    np.testing.assert_allclose(tri["quats"][0], sc.quats[0], atol=0)
    np.testing.assert_allclose(tri["scales"][0], sc.scales[0], atol=0)


def test_thresholds_of_sec_5_2():
    cams = synth.hemisphere_cameras(3, 4.0, 200, 160)
    sv, mom = _fake_sv(cams, np.zeros(3), np.eye(3) * 1e-3)
    sc = scene_of([[0, 0, 0]], [[1, 0, 0, 0]], [[0.03, 0.03, 0.03]], [0.5])
    sv1 = dict(sv)
    sv1["flags"] = sv["flags"].copy()
    sv1["flags"][1:] = oracle.VF_FEW_PIX
    assert oracle.triangulate(sc, cams, sv1, mom, np.ones((3, 1), np.uint8))["status"][0] & oracle.ST_FEW_VIEWS
    mom2 = mom.copy()
    mom2[..., oracle.S_W] = 3e-4
    assert oracle.triangulate(sc, cams, sv, mom2, np.ones((3, 1), np.uint8))["status"][0] & oracle.ST_LOW_ALPHA
    mom3 = mom.copy()
    mom3[..., oracle.S_N] = [[1], [1], [0]]
    assert oracle.triangulate(sc, cams, sv, mom3, np.ones((3, 1), np.uint8))["status"][0] & oracle.ST_FEW_PIX
    # per-view solve thresholds
    m = np.zeros((1, 4, 16))
    m[0, 0, [oracle.S_W, oracle.S_N]] = [1e-4, 5]
    m[0, 1, [oracle.S_W, oracle.S_N]] = [0.5, 1]
    m[0, 2, [oracle.S_W, oracle.S_N, oracle.S_UXUX, oracle.S_UYUY]] = [0.5, 5, 1e-7, 1e-7]
    m[0, 3, [oracle.S_W, oracle.S_N, oracle.S_UXUX, oracle.S_UYUY]] = [0.5, 5, 2.0, 3.0]
    out = oracle.solve_views(m, np.zeros((1, 4, 2)), np.zeros((1, 4, 3)), np.ones((1, 4), np.uint8))
    assert out["flags"][0, 0] & oracle.VF_LOW_ALPHA
    assert out["flags"][0, 1] & oracle.VF_FEW_PIX
    assert out["flags"][0, 2] & oracle.VF_SINGULAR
    assert out["flags"][0, 3] == oracle.VF_OK
    # near-singular V1 independently of scale: pixels on one line (a single
    # column) make V1 exactly singular, however many pixels there are
    xs = np.zeros(9)
    ys = np.arange(9.0) - 4.0
    w = np.linspace(0.2, 0.6, 9)
    rec = np.zeros((1, 1, 16))
    rec[0, 0, oracle.S_W] = w.sum()
    rec[0, 0, oracle.S_UX], rec[0, 0, oracle.S_UY] = (w * xs).sum(), (w * ys).sum()
    rec[0, 0, oracle.S_UXUX], rec[0, 0, oracle.S_UXUY] = (w * xs * xs).sum(), (w * xs * ys).sum()
    rec[0, 0, oracle.S_UYUY] = (w * ys * ys).sum()
    rec[0, 0, oracle.S_N] = 9
    line = rec.copy()
    line[0, 0, oracle.S_UXUX] += 1e-7 * line[0, 0, oracle.S_UYUY]   # FP32-sized residue
    out = oracle.solve_views(line, np.zeros((1, 1, 2)), np.zeros((1, 1, 3)), np.ones((1, 1), np.uint8))
    assert out["flags"][0, 0] & oracle.VF_SINGULAR
    strip = rec.copy()
    strip[0, 0, oracle.S_UXUX] = 0.25 * strip[0, 0, oracle.S_W]       # two columns +-0.5 px
    out = oracle.solve_views(strip, np.zeros((1, 1, 2)), np.zeros((1, 1, 3)), np.ones((1, 1), np.uint8))
    assert out["flags"][0, 0] == oracle.VF_OK


# ----------------------------------------------------------------- P10: exact recovery end to end
def _monge(S, Sp):
    """Optimal-transport (Monge) linear map between centred Gaussians N(0,S)
    and N(0,Sp): A = S^-1/2 (S^1/2 Sp S^1/2)^1/2 S^-1/2, so A S A^T = Sp."""
    def sqrtm(M):
        w, U = np.linalg.eigh(M)
        return U @ np.diag(np.sqrt(w)) @ U.T
    Sh = sqrtm(S)
    Shi = np.linalg.inv(Sh)
    return Shi @ sqrtm(Sh @ Sp @ Sh) @ Shi


@pytest.mark.parametrize("V", [2, 3, 4, 6, 8])
def test_p10_exact_recovery_single_gaussian(V):
    rng = np.random.default_rng(100 + V)
    cams = synth.hemisphere_cameras(V, 3.0, 160, 160, fov_x_deg=50.0)
    for trial in range(20 if V <= 4 else 8):
        mu = rng.uniform(-0.15, 0.15, 3)
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        q[0] = abs(q[0])
        s = np.sort(rng.uniform(0.06, 0.12, 3))[rng.permutation(3)]
        rot = Rotation.from_rotvec(rng.standard_normal(3) / math.sqrt(3) * math.radians(rng.uniform(0, 30)))
        t = rng.standard_normal(3)
        t *= rng.uniform(0, 0.3) / np.linalg.norm(t)
        mu_n = mu + t
        R_n = rot.as_matrix() @ Rotation.from_quat([*q[1:], q[0]]).as_matrix()
        qn = Rotation.from_matrix(R_n).as_quat()[[3, 0, 1, 2]]
        qn *= np.sign(qn[0])
        sc = scene_of([mu], [q], [s], [0.9])
        moved = scene_of([mu_n], [qn], [s], [0.9])
        g = oracle.geometry(sc, cams)
        cov0, _ = oracle.project64(sc, cams)
        cov1, _ = oracle.project64(moved, cams)
        disp = np.zeros((V, 160, 160, 2))
        cc, rr = np.meshgrid(np.arange(160.0), np.arange(160.0))
        for v, cam in enumerate(cams):
            S0 = np.array([[cov0[v, 0, 0], cov0[v, 0, 1]], [cov0[v, 0, 1], cov0[v, 0, 2]]])
            S1 = np.array([[cov1[v, 0, 0], cov1[v, 0, 1]], [cov1[v, 0, 1], cov1[v, 0, 2]]])
            A = _monge(S0, S1)
            x1, _ = pinhole(cam, moved.means[0].astype(np.float64))
            b = x1 - A @ g.mu[v, 0].astype(np.float64)
            disp[v, ..., 0] = A[0, 0] * cc + A[0, 1] * rr + b[0] - cc
            disp[v, ..., 1] = A[1, 0] * cc + A[1, 1] * rr + b[1] - rr
        # FP64 tracks straight into the FP64 oracle
        r = oracle.motion_transfer(sc, cams, disp, np.ones((V, 160, 160), np.uint8))
        tri = r["tri"]
        np.testing.assert_allclose(tri["means"][0], moved.means[0], atol=1e-9)
        if V == 2:
            assert tri["status"][0] == oracle.ST_POS | oracle.ST_NEG_EIG
            continue
        assert tri["status"][0] == oracle.ST_POS | oracle.ST_COV, (trial, tri["status"][0], r["sv"]["flags"][:, 0])
        dq = abs(float(np.dot(tri["quats"][0], moved.quats[0].astype(np.float64) /
                              np.linalg.norm(moved.quats[0].astype(np.float64)))))
        ang = math.degrees(2 * math.acos(min(1.0, dq)))
        # FP64 recovery; the 3-view covariance system can have a condition
        # number near 1e8, hence 1e-5 degrees rather than machine precision
        assert ang < 1e-5, ang
        np.testing.assert_allclose(tri["scales"][0], moved.scales[0], rtol=1e-8)


# ----------------------------------------------------------------- P11: invariants
def test_p11_identity_and_constant_shift():
    wl = synth.make_workload("small", seed=21, n=800, with_tracks=False)
    V = len(wl.cams)
    zero = np.zeros_like(wl.disp)
    r = oracle.motion_transfer(wl.scene, wl.cams, zero, None)
    sv = r["sv"]
    ok = sv["flags"] == oracle.VF_OK
    np.testing.assert_array_equal(sv["A"][ok], np.broadcast_to(np.eye(2), sv["A"][ok].shape))
    np.testing.assert_array_equal(sv["c"][ok], 0.0)
    tri = r["tri"]
    pos = (tri["status"] & oracle.ST_POS) > 0
    assert pos.mean() > 0.5
    np.testing.assert_allclose(tri["means"][pos], wl.scene.means[pos], atol=2e-5)
    cv = (tri["status"] & oracle.ST_COV) > 0
    np.testing.assert_allclose(tri["scales"][cv], wl.scene.scales[cv], rtol=2e-3)
    shift = np.array([[1.5, -0.5], [0.0, 2.0], [-1.0, -1.0], [0.7, 0.3]])[:V]
    d = np.broadcast_to(shift[:, None, None, :], wl.disp.shape).astype(np.float32)
    r2 = oracle.motion_transfer(wl.scene, wl.cams, d, None)
    sv2 = r2["sv"]
    ok2 = sv2["flags"] == oracle.VF_OK
    np.testing.assert_allclose(sv2["A"][ok2], np.broadcast_to(np.eye(2), sv2["A"][ok2].shape), atol=1e-9)
    cvec = np.broadcast_to(shift[:, None, :], sv2["c"].shape)
    np.testing.assert_allclose(sv2["c"][ok2], cvec[ok2], atol=1e-9)


# ----------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_mistakes(monkeypatch):
    """A dropped term or swapped index in the oracle's solve must fail P6."""
    A_true = np.array([[1.08, -0.05], [0.03, 0.95]])
    b_true = np.array([3.0, -1.5])
    fn = lambda c, r: np.stack([A_true[0, 0] * c + A_true[0, 1] * r + b_true[0] - c,
                                A_true[1, 0] * c + A_true[1, 1] * r + b_true[1] - r], -1)
    sc, cam, d = _single_gaussian_frame(3, fn)
    good = oracle.v1_v2

    def transposed(mom):
        V1, V2 = good(mom)
        V2 = V2.copy()
        V2[..., 0:2, :] = np.swapaxes(V2[..., 0:2, :], -1, -2)
        return V1, V2

    def dropped(mom):
        V1, V2 = good(mom)
        V1 = V1.copy()
        V1[..., 0, 2] = V1[..., 2, 0] = 0.0
        return V1, V2

    for bad in (transposed, dropped):
        monkeypatch.setattr(oracle, "v1_v2", bad)
        r = oracle.motion_transfer(sc, [cam], d.astype(np.float64), np.ones((1, 96, 96), np.uint8))
        mu = r["geom"].mu[0, 0].astype(np.float64)
        A = r["sv"]["A"][0, 0]
        b = r["sv"]["mu_new"][0, 0] - A @ mu
        assert not (np.allclose(A, A_true, atol=2e-7) and np.allclose(b, b_true, atol=5e-5))
    monkeypatch.setattr(oracle, "v1_v2", good)


# ----------------------------------------------------------------- generator
def test_generator_is_seeded_and_shaped():
    a = synth.make_workload("small", seed=2)
    b = synth.make_workload("small", seed=2)
    assert a.disp.tobytes() == b.disp.tobytes() and a.scene.means.tobytes() == b.scene.means.tobytes()
    c = synth.make_workload("small", seed=3)
    assert a.disp.tobytes() != c.disp.tobytes()
    assert a.disp.shape == (4, 128, 128, 2) and a.vis.shape == (4, 128, 128)
    assert np.all(a.scene.quats[:, 0] >= 0)
    assert np.all((a.scene.opacity > 0.1) & (a.scene.opacity < 0.9))
    assert np.all((a.scene.scales >= 0.01 - 1e-7) & (a.scene.scales <= 0.05 + 1e-7))


def test_generator_outliers_visibility_and_cap():
    rng = np.random.default_rng(0)
    cams = synth.hemisphere_cameras(2, 6.0, 320, 180)
    sc = synth.random_gaussians(rng, 5000, domain="ball", radius=2.0)
    mo = synth.body_field_motion(rng, sc, cams, max_angle_deg=30, max_trans=0.3, cap_px=25.0)
    for cam in cams:
        a, _ = synth._pinhole(cam, sc.means.astype(np.float64))
        b, _ = synth._pinhole(cam, mo.means.astype(np.float64))
        assert np.abs(b - a).max() <= 25.0 * 1.05
    disp, vis = synth.proxy_tracks(rng, cams, mo.field, radius=2.0, noise_px=1.0, outlier_rate=0.05,
                                   vis_rate=0.9)
    n = vis.size
    p = vis.mean()
    assert abs(p - 0.9) < 3 * math.sqrt(0.09 / n) + 1e-3
    big = (np.linalg.norm(disp, axis=-1) > 60).mean()
    assert 0.02 < big < 0.06


# ----------------------------------------------------------------- static-pixel slots (Sec. 4.5.2)
@pytest.mark.parametrize("disp,static", [((0.5, 0.0), True), ((0.0, -0.5), True),
                                         ((np.nextafter(np.float32(1), np.float32(0)), 0.0), True),
                                         ((1.0, 0.0), False), ((0.0, -1.0), False), ((0.8, 0.7), False)])
def test_static_slots_count_and_alpha(disp, static):
    """A covered pixel whose track moves less than 1 px adds 1 to slot 13
    and its alpha (not the weight alpha T) to slot 14; at |d| = 1 it is not
    static.  Two Gaussians front to back make alpha and w differ for the one
    behind (w = alpha (1 - alpha_front)), so a weight in slot 14 fails, and
    the boundary cases fail a <= in place of <."""
    cam = axis_camera(4.0)
    sc = scene_of([[0, 0, 0.5], [0, 0, -0.5]], [[1, 0, 0, 0]] * 2, [[0.1, 0.1, 0.1], [0.12, 0.12, 0.12]],
                  [0.6, 0.8])
    px = py = 31
    g, cov, conic, r = _single_pixel_run(sc, cam, px, py, disp=disp)
    m = r["mom"][0]
    al = []
    for i in range(2):
        mu = g.mu[0, i].astype(np.float64)
        d = np.array([px - mu[0], py - mu[1]])
        cn = conic[0, i]
        power = -0.5 * (cn[0] * d[0] ** 2 + cn[2] * d[1] ** 2) - cn[1] * d[0] * d[1]
        al.append(min(0.99, float(sc.opacity[i]) * math.exp(power)))
    assert m[1, oracle.S_N] == 1 and m[0, oracle.S_N] == 1
    if static:
        np.testing.assert_array_equal(m[:, oracle.S_STATN], [1.0, 1.0])
        np.testing.assert_allclose(m[1, oracle.S_STATA], al[1], rtol=1e-12)    # front: alpha = w
        np.testing.assert_allclose(m[0, oracle.S_STATA], al[0], rtol=1e-12)    # behind: alpha, not w
        assert abs(m[0, oracle.S_STATA] - m[0, oracle.S_W]) > 0.05
    else:
        np.testing.assert_array_equal(m[:, oracle.S_STATN], [0.0, 0.0])
        np.testing.assert_array_equal(m[:, oracle.S_STATA], [0.0, 0.0])
    # an invisible track adds nothing, static or not
    g, cov, conic, r = _single_pixel_run(sc, cam, px, py, disp=disp, vis=0)
    np.testing.assert_array_equal(r["mom"][0, :, :15], 0.0)


# ----------------------------------------------------------------- tile rectangle (Sec. 3.1, Eq. 1)
def test_tile_rectangle_closed_form():
    """An axis-aligned Gaussian off the optical axis: Eq. 1 gives
    Sigma_2D = J diag(s^2) J^T with J = [[f/z, 0, -f x/z^2], [0, f/z, -f y/z^2]]
    in closed form; the rectangle is the tiles met by the square of half
    side ceil(3 sqrt(lambda_max(Sigma_2D + 0.3 I))) about the centre.  The
    values are chosen away from every rounding boundary, so the FP32
    rectangle must equal this one exactly (one tile more or less fails)."""
    f, z, W = 200.0, 4.0, 256
    cam = synth.Camera(R=np.eye(3, dtype=np.float32), t=np.array([0, 0, z], np.float32), fx=f, fy=f,
                       cx=(W - 1) / 2, cy=(W - 1) / 2, W=W, H=W)
    for (x, y, sx, sy, sz) in [(0.3, -0.2, 0.2, 0.1, 0.05), (-0.43, 0.35, 0.04, 0.15, 0.1),
                               (0.13, 0.6, 0.3, 0.3, 0.02)]:
        sc = scene_of([[x, y, 0.0]], [[1, 0, 0, 0]], [[sx, sy, sz]], [0.5])
        g = oracle.geometry(sc, [cam])
        xf, yf = np.float64(np.float32(x)), np.float64(np.float32(y))
        s = np.asarray([sx, sy, sz], np.float32).astype(np.float64)
        a = (f / z) ** 2 * s[0] ** 2 + (f * xf / z ** 2) ** 2 * s[2] ** 2 + 0.3
        b = (f * xf / z ** 2) * (f * yf / z ** 2) * s[2] ** 2
        c = (f / z) ** 2 * s[1] ** 2 + (f * yf / z ** 2) ** 2 * s[2] ** 2 + 0.3
        lmax = 0.5 * (a + c) + math.sqrt(0.25 * (a - c) ** 2 + b * b)
        r3 = 3.0 * math.sqrt(lmax)
        assert abs(r3 - round(r3)) > 1e-3
        rad = math.ceil(r3)
        mu = np.array([f * xf / z + (W - 1) / 2, f * yf / z + (W - 1) / 2])
        np.testing.assert_allclose(g.mu[0, 0], mu, atol=1e-4)
        lo, hi = (mu - rad) / 16.0, (mu + rad) / 16.0
        assert np.all(np.abs(lo - np.round(lo)) > 1e-3) and np.all(np.abs(hi - np.round(hi)) > 1e-3)
        T = W // 16
        want = [max(0, math.floor(lo[0])), max(0, math.floor(lo[1])), min(T, math.floor(hi[0]) + 1),
                min(T, math.floor(hi[1]) + 1)]
        np.testing.assert_array_equal(g.rect[0, 0], want)


# ----------------------------------------------------------------- non-finite inputs
def test_nonfinite_gaussian_equals_removed_gaussian():
    """A Gaussian with a non-finite parameter is culled in every view, so the
    rest of the frame equals the frame without it (bit for bit: same lists,
    same sums); it reports status 256 and is copied."""
    wl = synth.make_workload("small", seed=31, n=600)
    bad = np.array([3, 50, 51, 200, 599])
    sc = synth.Scene(means=wl.scene.means.copy(), quats=wl.scene.quats.copy(), scales=wl.scene.scales.copy(),
                     opacity=wl.scene.opacity.copy(), rgb=wl.scene.rgb)
    sc.means[3, 1] = np.nan
    sc.quats[50, 0] = np.inf
    sc.scales[51, 2] = np.nan
    sc.opacity[200] = np.nan
    sc.means[599, 0] = -np.inf
    keep = np.setdiff1d(np.arange(sc.n), bad)
    sub = synth.Scene(means=wl.scene.means[keep], quats=wl.scene.quats[keep], scales=wl.scene.scales[keep],
                      opacity=wl.scene.opacity[keep], rgb=wl.scene.rgb[keep])
    r = oracle.motion_transfer(sc, wl.cams, wl.disp, wl.vis)
    r0 = oracle.motion_transfer(sub, wl.cams, wl.disp, wl.vis)
    tri, tri0 = r["tri"], r0["tri"]
    assert np.all(tri["status"][bad] & oracle.ST_NONFINITE)
    assert not np.any(tri["status"][bad] & (oracle.ST_POS | oracle.ST_COV))
    assert np.all(r["geom"].valid[:, bad] == 0)
    np.testing.assert_array_equal(tri["status"][keep], tri0["status"])
    np.testing.assert_array_equal(r["comp"]["mom"][:, keep], r0["comp"]["mom"])
    np.testing.assert_array_equal(tri["means"][keep], tri0["means"])
    np.testing.assert_array_equal(tri["quats"][keep], tri0["quats"])
    np.testing.assert_array_equal(tri["means"][bad], sc.means[bad].astype(np.float64))


def test_nonfinite_tracks_flag_exactly_the_views_they_reach():
    """A non-finite track poisons the sums of every (view, Gaussian) record
    its pixel feeds (visible and contributing); exactly those views get
    flag 32 and are left out of the multi-view update, and their Gaussians
    report status 256.  The records it feeds are found by compositing only
    the poisoned pixels."""
    wl = synth.make_workload("small", seed=32, n=800)
    disp = wl.disp.copy()
    pix = [(0, 40, 60), (1, 70, 20), (2, 64, 64), (3, 10, 100)]
    mask = np.zeros(wl.vis.shape, np.uint8)
    for v, y, x in pix:
        disp[v, y, x, 0] = np.nan
        mask[v, y, x] = 1
    vis = np.ones_like(wl.vis)
    r = oracle.motion_transfer(wl.scene, wl.cams, disp, vis)
    g = r["geom"]
    only = oracle.composite(wl.scene, wl.cams, g, r["conic"], r["lists"], wl.disp, vis, pixmask=mask)
    reached = only["mom"][..., oracle.S_N] > 0
    assert reached.sum() >= 4
    np.testing.assert_array_equal((r["sv"]["flags"] & oracle.VF_NONFINITE) > 0, reached)
    st = r["tri"]["status"]
    np.testing.assert_array_equal((st & oracle.ST_NONFINITE) > 0, reached.any(0))
    # the remaining views of those Gaussians still count as in any other frame
    clean = oracle.motion_transfer(wl.scene, wl.cams, wl.disp, vis)
    untouched = ~reached.any(0)
    assert np.isfinite(r["tri"]["means"]).all()
    np.testing.assert_array_equal(r["sv"]["flags"][:, untouched], clean["sv"]["flags"][:, untouched])
