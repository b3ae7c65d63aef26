"""Pins of the motion-regularisation oracle (oracle/regularize.py), CPU only:
the static rule at its boundaries, KNN against a brute-force distance sort,
the Euler convention against scipy's rotations, exact recovery of a uniform
change (median and mean of identical values), salt-and-pepper removal, and
what static and source-less Gaussians keep."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth
from oracle import regularize as rg


def test_static_rule_boundaries():
    V, N = 3, 8
    acc = np.zeros((V, N, 16), np.float32)
    # (pixels, static pixels) in views 0 and 1; view 2 empty
    cases = [((10, 10), (10, 10), True),    # > 9 pixels, 100% static, 2 views
             ((9, 9), (10, 10), False),     # 9 pixels is not "more than 9"
             ((10, 9), (10, 10), False),    # 90% is not "more than 90%"
             ((20, 19), (11, 10), True),    # 95% and 90.9%
             ((20, 19), (0, 0), False),     # one view only
             ((100, 91), (100, 91), True),
             ((100, 90), (100, 91), False),
             ((0, 0), (0, 0), False)]
    for i, ((n0, s0), (n1, s1), _) in enumerate(cases):
        acc[0, i, oracle.S_N], acc[0, i, oracle.S_STATN] = n0, s0
        acc[1, i, oracle.S_N], acc[1, i, oracle.S_STATN] = n1, s1
    np.testing.assert_array_equal(rg.static_mask(acc), [c[2] for c in cases])


def test_knn_matches_brute_force():
    rng = np.random.default_rng(0)
    pts = rng.uniform(-1, 1, (600, 3)).astype(np.float32)
    src = np.nonzero(rng.random(600) < 0.6)[0]
    qry = np.arange(600)
    idx, dist = rg.knn(pts, src, qry, 8)
    p64 = pts.astype(np.float64)
    d2 = ((p64[qry][:, None, :] - p64[src][None, :, :]) ** 2).sum(-1)
    order = np.argsort(d2, axis=1, kind="stable")[:, :8]
    np.testing.assert_array_equal(idx, order)
    np.testing.assert_allclose(dist, np.sqrt(np.take_along_axis(d2, order, 1)), rtol=1e-12)


def test_knn_ties_by_index():
    """Exact duplicates (equal distances, also past the tree's first
    candidates): neighbours are the lowest indices among equal distances,
    as a stable brute-force sort orders them."""
    rng = np.random.default_rng(1)
    base = rng.uniform(-1, 1, (40, 3)).astype(np.float32)
    pts = base[rng.integers(0, 40, 400)]          # every position about 10 times
    pts[:30] = pts[0]                              # one position 30+ times
    src = np.nonzero(rng.random(400) < 0.7)[0]
    src = np.union1d(src, np.arange(30))
    qry = np.arange(400)
    idx, dist = rg.knn(pts, src, qry, 8)
    p64 = pts.astype(np.float64)
    d2 = ((p64[qry][:, None, :] - p64[src][None, :, :]) ** 2).sum(-1)
    order = np.argsort(d2, axis=1, kind="stable")[:, :8]
    np.testing.assert_array_equal(idx, order)
    assert (dist[:30] == 0).all()


def test_euler_convention_against_scipy():
    rng = np.random.default_rng(1)
    R = Rotation.random(200, random_state=2)
    M = R.as_matrix()
    e = rg.euler_zyx(M)
    # scipy 'ZYX' (intrinsic) gives (psi, theta, phi) for Rz(psi) Ry(theta) Rx(phi)
    ref = R.as_euler("ZYX")
    np.testing.assert_allclose(e[:, ::-1], ref, atol=1e-12)
    np.testing.assert_allclose(rg.rot_zyx(e), M, atol=1e-12)


def test_uniform_change_is_recovered_exactly():
    c = synth.make_reg_case(3000, seed=3, uniform=True)
    m, q, s, reg = rg.regularize(c.scene.means, c.scene.quats, c.scene.scales, c.means1, c.quats1, c.scales1,
                                 c.status, c.acc)
    static = rg.static_mask(c.acc)
    moved = ~static
    # every non-static Gaussian (solved: median of identical changes;
    # unsolved: their mean) ends at the ground truth
    assert ((reg[moved] & (rg.RG_FILTERED | rg.RG_PROPAGATED)) > 0).all()
    np.testing.assert_allclose(m[moved], c.truth["means"][moved], atol=2e-6)
    # rotations as matrices (the FP32-stored inputs limit this to ~1e-7)
    np.testing.assert_allclose(oracle.quat_to_rot(q[moved]), oracle.quat_to_rot(c.truth["quats"][moved]),
                               atol=2e-6)
    np.testing.assert_allclose(s[moved], c.scene.scales[moved], rtol=1e-6)
    # static Gaussians keep the first frame exactly
    np.testing.assert_array_equal(m[static], c.scene.means[static])
    np.testing.assert_array_equal(q[static], c.scene.quats[static])
    assert (reg[static] == rg.RG_STATIC).all()


def test_salt_and_pepper_outliers_are_removed():
    c = synth.make_reg_case(4000, seed=4, noise=0.0, outlier_frac=0.05)
    # truth-consistent changes except for the outliers: the filtered result
    # of almost every solved Gaussian is close to the truth
    m, q, s, reg = rg.regularize(c.scene.means, c.scene.quats, c.scene.scales, c.means1, c.quats1, c.scales1,
                                 c.status, c.acc)
    solved = (reg & rg.RG_FILTERED) > 0
    err_in = np.linalg.norm(c.means1[solved] - c.truth["means"][solved], axis=-1)
    err_out = np.linalg.norm(m[solved] - c.truth["means"][solved], axis=-1)
    assert (err_in > 0.05).mean() > 0.03          # the input has outliers
    assert (err_out > 0.05).mean() < 0.002        # the median removed them
    # a plain mean would not: the planted mistake (mean instead of median)
    src = np.nonzero(solved)[0]
    d = rg.deltas(c.scene.means, c.scene.quats, c.scene.scales, c.means1, c.quats1, c.scales1)
    idx, _ = rg.knn(c.scene.means, src, src)
    m_mean = c.scene.means[src] + d[src][idx].mean(1)[:, :3]
    assert (np.linalg.norm(m_mean - c.truth["means"][src], axis=-1) > 0.05).mean() > 0.05


def test_no_sources_leaves_everything_unchanged():
    c = synth.make_reg_case(500, seed=5)
    status = np.full_like(c.status, 4)
    m, q, s, reg = rg.regularize(c.scene.means, c.scene.quats, c.scene.scales, c.means1, c.quats1, c.scales1,
                                 status, c.acc)
    static = rg.static_mask(c.acc)
    np.testing.assert_array_equal(m, c.scene.means)
    np.testing.assert_array_equal(s, c.scene.scales)
    np.testing.assert_array_equal(reg, np.where(static, rg.RG_STATIC, 0))


def test_median_of_eight_is_mean_of_middle_pair():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((100, 8))
    xs = np.sort(x, 1)
    np.testing.assert_allclose(np.median(x, 1), 0.5 * (xs[:, 3] + xs[:, 4]), rtol=0, atol=0)
