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


def _propagation_scene():
    """One unsolved target at the origin and 8 clusters of 8 solved
    Gaussians.  Cluster i sits on a ray at 45 i degrees: its seed s_i at
    radius 1 + 0.001 i (the 8 seeds are the target's 8 nearest solved
    Gaussians, nearest first by i) and 7 companions 0.01-0.07 further out on
    the ray (each cluster is its own members' 8-neighbourhood; clusters are
    0.76 apart).  The companions move by c_i, the seed by c_i + 0.5 (a raw
    outlier), so the filtered change of every member is c_i exactly: the
    median of 8 values of which 7 equal c_i."""
    base = np.array([1.0, -2.0, 0.5, 0.3, -0.2, 0.4, 0.1, 0.05, -0.08])
    c = np.stack([0.01 * i * i * base for i in range(8)])          # asymmetric in i
    pts, chg, role = [np.zeros(3)], [np.zeros(9)], [-1]
    for i in range(8):
        u = np.array([np.cos(np.pi / 4 * i), np.sin(np.pi / 4 * i), 0.0])
        r = 1.0 + 0.001 * i
        pts.append(r * u)
        chg.append(c[i] + 0.5)
        role.append(i)
        for j in range(1, 8):
            pts.append((r + 0.01 * j) * u)
            chg.append(c[i])
            role.append(i)
    pts, chg, role = np.array(pts), np.array(chg), np.array(role)
    n = len(pts)
    rng = np.random.default_rng(9)
    q0 = rng.standard_normal((n, 4))
    q0 /= np.linalg.norm(q0, axis=1, keepdims=True)
    q0[q0[:, 0] < 0] *= -1
    s0 = np.full((n, 3), 0.1)
    R1 = rg.rot_zyx(chg[:, 3:6]) @ oracle.quat_to_rot(q0)
    q1 = oracle.rot_to_quat(R1)
    status = np.full(n, oracle.ST_POS | oracle.ST_COV, np.uint32)
    status[0] = oracle.ST_FEW_VIEWS                                   # the target
    acc = np.zeros((2, n, 16), np.float32)                            # nothing static
    return dict(m0=pts, q0=q0, s0=s0, m1=pts + chg[:, 0:3], q1=q1, s1=s0 + chg[:, 6:9], status=status,
                acc=acc, c=c, outlier=c + 0.5)


def _target_change(sc):
    m, q, s, reg = rg.regularize(sc["m0"], sc["q0"], sc["s0"], sc["m1"], sc["q1"], sc["s1"], sc["status"],
                                 sc["acc"])
    assert reg[0] == rg.RG_PROPAGATED and (reg[1:] == rg.RG_FILTERED).all()
    e = rg.euler_zyx(oracle.quat_to_rot(q[0:1]) @ oracle.quat_to_rot(sc["q0"][0:1]).swapaxes(-1, -2))[0]
    return np.concatenate([m[0] - sc["m0"][0], e, s[0] - sc["s0"][0]])


def test_propagation_is_mean_of_filtered_neighbour_changes():
    """Sec. 4.5.2: an unsolved Gaussian takes the component-wise mean of its
    K = 8 nearest solved Gaussians' filtered (median) changes; the expected
    value is the mean of the 8 clusters' c_i, written out by hand."""
    sc = _propagation_scene()
    want = sc["c"].mean(0)
    got = _target_change(sc)
    np.testing.assert_allclose(got, want, atol=1e-9)
    # the construction separates the readings a mistake would take
    assert np.abs(np.median(sc["c"], 0) - want).max() > 0.01        # median instead of mean
    assert np.abs(sc["outlier"].mean(0) - want).max() > 0.1         # raw instead of filtered
    assert np.abs(sc["c"][:4].mean(0) - want).max() > 0.01          # K = 4


@pytest.mark.parametrize("mistake", ["median", "raw", "k4"])
def test_propagation_pin_catches_planted_mistakes(monkeypatch, mistake):
    sc = _propagation_scene()
    if mistake == "median":
        monkeypatch.setattr(rg, "propagate", lambda vals: np.median(vals, axis=1))
    elif mistake == "raw":
        # each solved Gaussian passes on its own raw change (its nearest
        # neighbour is itself) instead of the filtered one
        monkeypatch.setattr(rg, "median_filter", lambda vals: vals[:, 0])
    else:
        monkeypatch.setattr(rg, "K", 4)
    got = _target_change(sc)
    assert not np.allclose(got, sc["c"].mean(0), atol=1e-6)
