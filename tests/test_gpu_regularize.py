"""GPU parity of tg_regularize (motion regularisation, Sec. 4.5) against the
oracle on the same seeded inputs: classification (static / filtered /
propagated / unchanged) bit-exact; means within 1e-5 plus one FP32 ulp of
the coordinate (the output positions are FP32, so a scene far from the origin
carries one rounding of its own size), rotation matrices within 1e-5 and
scales within 1e-5 relative (the kernel stores the changes in FP32; medians
and means are continuous in them)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import log
from oracle import regularize as rg

pytestmark = pytest.mark.gpu

CASES = {
    "default": dict(n=5000, views=4, seed=7),
    "uniform": dict(n=3000, views=3, seed=8, uniform=True),
    "dense_outliers": dict(n=20000, views=5, seed=9, outlier_frac=0.15, unsolved_frac=0.3),
    "few_sources": dict(n=4000, views=4, seed=10, unsolved_frac=0.97, posonly_frac=0.0),
    "large": dict(n=200_000, views=6, seed=11),
    # a scene 1000 units from the origin: the FP32 screens' roundings are
    # largest relative to the distances
    "far_offset": dict(n=20000, views=4, seed=13, offset=(1000.0, -750.0, 500.0)),
    # a fifth of the Gaussians share another's position: equal distances,
    # neighbours decided by index
    "duplicates": dict(n=20000, views=4, seed=14, dup_frac=0.2),
    # only a shell of the ball solved: queries in the interior are far from
    # every solved Gaussian (long searches, the screens' bounds near their
    # thresholds for many points at once)
    "shell": dict(n=60000, views=4, seed=15, shell=1.8, unsolved_frac=0.0, static_frac=0.0),
}


def _run_gpu(c, no_sources=False):
    from paper_2604_02586_amd import api
    dev = torch.device("cuda:0")
    t = lambda x, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(x)).to(dev, dt).contiguous()
    n = c.scene.n
    g_ref = api.GaussianTensors(t(c.scene.means), t(c.scene.quats), t(c.scene.scales), t(c.scene.opacity))
    g_upd = api.GaussianTensors(t(c.means1), t(c.quats1), t(c.scales1), g_ref.opacity)
    g_out = api.GaussianTensors(torch.empty_like(g_ref.means), torch.empty_like(g_ref.quats),
                                torch.empty_like(g_ref.scales), g_ref.opacity)
    status = np.full_like(c.status, 4) if no_sources else c.status
    st = torch.as_tensor(status.view(np.int32)).to(dev)
    acc = t(c.acc)
    reg = torch.empty(n, dtype=torch.int32, device=dev)
    api.regularize(g_ref, g_upd, st, acc, api.default_params(), g_out, reg)
    torch.cuda.synchronize()
    h = lambda x: x.cpu().numpy()
    return h(g_out.means), h(g_out.quats), h(g_out.scales), h(reg).view(np.uint32), status


@pytest.mark.parametrize("case", list(CASES))
def test_regularize_matches_oracle(case):
    c = synth.make_reg_case(**CASES[case])
    log(f"[{case}] n={c.scene.n}")
    m, q, s, reg, status = _run_gpu(c)
    om, oq, os_, oreg = rg.regularize(c.scene.means, c.scene.quats, c.scene.scales, c.means1, c.quats1, c.scales1,
                                      status, c.acc)
    np.testing.assert_array_equal(reg, oreg)
    moved = (oreg & (rg.RG_FILTERED | rg.RG_PROPAGATED)) > 0
    err_m = np.abs(m.astype(np.float64) - om)
    dm = err_m.max() if m.size else 0.0
    Rg = oracle.quat_to_rot(q[moved].astype(np.float64))
    Ro = oracle.quat_to_rot(oq[moved])
    dr = np.abs(Rg - Ro).max() if moved.any() else 0.0
    ds = np.abs(s[moved] / os_[moved] - 1).max() if moved.any() else 0.0
    log(f"[{case}] filtered {int(((oreg & 2) > 0).sum())} propagated {int(((oreg & 4) > 0).sum())} "
        f"static {int((oreg == 1).sum())}; max |dmu| {dm:.2e}, |dR| {dr:.2e}, |dS/S| {ds:.2e}")
    assert (err_m <= 1e-5 + 2.0 ** -23 * np.abs(om)).all() and dr <= 1e-5 and ds <= 1e-5
    assert (q[moved][:, 0] >= 0).all()
    # everything that does not move is copied bit-exactly
    keep = ~moved
    np.testing.assert_array_equal(m[keep], c.scene.means[keep])
    np.testing.assert_array_equal(q[keep], c.scene.quats[keep])
    np.testing.assert_array_equal(s[keep], c.scene.scales[keep])


def test_no_sources_moves_nothing():
    c = synth.make_reg_case(2000, views=3, seed=12)
    m, q, s, reg, status = _run_gpu(c, no_sources=True)
    np.testing.assert_array_equal(m, c.scene.means)
    np.testing.assert_array_equal(q, c.scene.quats)
    np.testing.assert_array_equal(reg, np.where(rg.static_mask(c.acc), rg.RG_STATIC, 0))
