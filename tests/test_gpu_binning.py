"""GPU binning (tg_bin_sort) against the oracle's depth order and coarse-bin
lists, bit-exact, on both emission paths: the direct placement (at most 256
coarse bins per view: per-block counts per bin, one scan, an in-LDS stable
sort by bin) and the general path (more bins per view: keys written in depth
order, then a stable radix sort over the bin bits).  Also the overflow
protocol: a capacity below the pair count sets the flag and reports the
count, and the retry with that count reproduces the lists."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import log

pytestmark = pytest.mark.gpu

CASES = {
    # 120 x 68 tiles -> 15 x 9 = 135 coarse bins per view: direct placement
    "direct_1080p": dict(name="small", seed=21, n=6000, views=3, width=1920, height=1080),
    # 33 x 9 = 297 coarse bins per view: general path
    "general_wide": dict(name="small", seed=22, n=3000, views=2, width=4200, height=1100),
    # 163 x 38 tiles -> 21 x 5 = 105 coarse bins per view: direct placement
    # with 8-byte coarse rectangles (more than 16 bins across)
    "direct_wide": dict(name="small", seed=24, n=4000, views=2, width=2600, height=600),
    # ragged tiles and bins, many Gaussians per bin
    "direct_dense": dict(name="medium", seed=23, n=40000, views=4, width=420, height=300),
}


def _bins_per_view(cams):
    return [((c.W + 15) // 16 + 7) // 8 * (((c.H + 15) // 16 + 7) // 8) for c in cams]


def _check(wl, mt):
    from paper_2604_02586_amd import api
    geom = oracle.geometry(wl.scene, wl.cams)
    V, N = geom.key.shape
    order = mt.bins.order.cpu().numpy().view(np.uint32)
    for v, o in enumerate(oracle.depth_order(geom)):
        np.testing.assert_array_equal(order[v, :o.size], o)
    starts, ids = oracle.cell_lists(geom, wl.cams, 8)
    assert int(mt.bins.n_pairs.item()) == ids.size
    assert int(mt.bins.overflow.item()) == 0
    cell_ids = mt.bins.cell_ids.cpu().numpy().view(np.uint32)
    rg = mt.bins.cell_ranges.cpu().numpy().view(np.uint32).reshape(-1, 2)
    assert rg.shape[0] == starts.size - 1
    for c in range(rg.shape[0]):
        a, b = int(starts[c]), int(starts[c + 1])
        assert rg[c, 1] - rg[c, 0] == b - a, c
        np.testing.assert_array_equal(cell_ids[rg[c, 0]:rg[c, 1]], ids[a:b])
    # the per-tile lists expanded from the bins equal the brute-force ones
    tids, tr = api.bin_expand(mt.splats, mt.bins, N, wl.cams, mt.params)
    tids = tids.cpu().numpy().view(np.uint32)
    tr = tr.cpu().numpy().view(np.uint32)
    ts, tl = oracle.cell_lists(geom, wl.cams, 1)
    assert tids.size == tl.size
    for t in range(tr.shape[0]):
        np.testing.assert_array_equal(tids[tr[t, 0]:tr[t, 1]], tl[ts[t]:ts[t + 1]])
    return ids.size


@pytest.mark.parametrize("case", list(CASES))
def test_bin_lists_bit_exact(case):
    from paper_2604_02586_amd import api
    kw = dict(CASES[case])
    wl = synth.make_workload(kw.pop("name"), **kw)
    log(f"[{case}] bins per view {_bins_per_view(wl.cams)[0]}")
    dev = torch.device("cuda:0")
    mt = api.MotionTransfer(wl.cams, wl.scene.n, dev)
    mt.preprocess(api.GaussianTensors.from_scene(wl.scene, dev))
    mt.bin_sort()
    torch.cuda.synchronize()
    n = _check(wl, mt)
    log(f"[{case}] {n} pairs bit-exact")


def test_overflow_then_retry():
    from paper_2604_02586_amd import api
    kw = dict(CASES["direct_1080p"])
    wl = synth.make_workload(kw.pop("name"), **kw)
    dev = torch.device("cuda:0")
    mt = api.MotionTransfer(wl.cams, wl.scene.n, dev, capacity=1024)
    mt.preprocess(api.GaussianTensors.from_scene(wl.scene, dev))
    mt.bin_sort(check_overflow=False)
    torch.cuda.synchronize()
    need = int(mt.bins.n_pairs.item())
    assert int(mt.bins.overflow.item()) == 1 and need > 1024
    # no list is published on overflow
    assert not mt.bins.cell_ranges.cpu().numpy().any()
    mt.bin_sort(check_overflow=True)   # re-sizes from the reported count
    torch.cuda.synchronize()
    assert _check(wl, mt) == need


def _axis_cams(W=256, H=192, f=500.0):
    # identity rotation and no depth offset: the depth key is the bits of mu_z
    return [synth.Camera(R=np.eye(3, dtype=np.float32), t=np.array([tx, 0.0, 0.0], np.float32), fx=f, fy=f,
                         cx=(W - 1) / 2, cy=(H - 1) / 2, W=W, H=H) for tx in (0.0, 0.3)]


def _axis_scene(rng, zs):
    n = zs.size
    u = rng.uniform(-0.15, 0.15, (n, 2)).astype(np.float32)
    means = np.concatenate([u * zs[:, None], zs[:, None]], 1).astype(np.float32)
    sc = synth.random_gaussians(rng, n)
    return synth.Scene(means=means, quats=sc.quats, scales=sc.scales, opacity=sc.opacity, rgb=sc.rgb)


DEPTH_CASES = {
    # one top key byte (0x40) and culled sentinels, no ordinary key whose low
    # 24 bits are all ones: the last radix pass is skipped
    "one_top_digit": lambda rng: rng.uniform(4.0, 7.9, 6000),
    # the same plus depths whose low 24 bits are all ones (7.99999952 =
    # 0x40FFFFFF), which tie with the sentinel below the top byte: the last
    # pass must run
    "tie_with_sentinel": lambda rng: np.concatenate([rng.uniform(4.0, 7.9, 6000),
                                                     np.full(7, np.float32(7.99999952))]),
    # two top bytes (0x40, 0x41): the last pass must run
    "two_top_digits": lambda rng: rng.uniform(4.0, 12.0, 6000),
}


@pytest.mark.parametrize("case", list(DEPTH_CASES))
def test_depth_order_with_culled_sentinels(case):
    """Depth keys crafted around the radix sort's skipped last pass: valid
    keys with one or two top bytes, culled Gaussians (behind the near plane,
    key 0xFFFFFFFF) mixed in at random indices; the order of the valid ones
    bit-exact and every culled one after them, by index."""
    from paper_2604_02586_amd import api
    rng = np.random.default_rng(61)
    zs = DEPTH_CASES[case](rng).astype(np.float32)
    culled = rng.random(zs.size) < 0.1
    culled[6000:] = False              # the crafted depths stay valid
    zs[culled] = np.float32(0.1)
    perm = rng.permutation(zs.size)
    zs, culled = zs[perm], culled[perm]
    scene = _axis_scene(rng, zs)
    cams = _axis_cams()
    wl = synth.Workload(name=case, scene=scene, cams=cams, motion=None,
                        disp=np.zeros((2, 192, 256, 2), np.float32), vis=np.ones((2, 192, 256), np.uint8))
    dev = torch.device("cuda:0")
    mt = api.MotionTransfer(cams, scene.n, dev)
    mt.preprocess(api.GaussianTensors.from_scene(scene, dev))
    mt.bin_sort()
    torch.cuda.synchronize()
    key = mt.splats.key.cpu().numpy().view(np.uint32)
    if case == "tie_with_sentinel":
        assert ((key != 0xFFFFFFFF) & ((key & 0xFFFFFF) == 0xFFFFFF)).sum() == 2 * 7
    geom = oracle.geometry(scene, cams)
    order = mt.bins.order.cpu().numpy().view(np.uint32)
    for v, o in enumerate(oracle.depth_order(geom)):
        np.testing.assert_array_equal(order[v, :o.size], o)
        tail = np.nonzero(~geom.valid[v].astype(bool))[0].astype(np.uint32)
        np.testing.assert_array_equal(order[v, o.size:], tail)
    log(f"[{case}] {int(culled.sum())} culled; depth order bit-exact")
    _check(wl, mt)
