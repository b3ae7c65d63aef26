"""GPU parity of tg_splat_accumulate_batch: several Gaussian sets of
different size, view count and resolution in one launch, each with several
frames of tracks sharing its alpha T.  Every frame's accumulators match the
oracle's compositing of that frame (same tolerance as the single-frame
path), and the batched launch equals separate single-frame launches up to
the order of FP32 atomic additions."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import compare_accumulators, log

pytestmark = pytest.mark.gpu

CLIPS = [
    dict(name="small", frames=1, n=700, views=2, width=64, height=48, seed=41),
    dict(name="large", frames=3, n=3000, views=3, width=150, height=100, seed=42),
    dict(name="medium", frames=2, n=1500, views=4, width=90, height=70, seed=43),
    dict(name="large", frames=4, n=2000, views=2, width=77, height=61, seed=44),
]


def _prepare(clip, dev):
    from paper_2604_02586_amd import api
    g = api.GaussianTensors.from_scene(clip.scene, dev)
    mt = api.MotionTransfer(clip.cams, clip.scene.n, dev)
    mt.preprocess(g)
    mt.bin_sort(check_overflow=True)
    return mt


@pytest.fixture(scope="module")
def batch():
    from paper_2604_02586_amd import api
    dev = torch.device("cuda:0")
    clips = [synth.make_clip(**c) for c in CLIPS]
    mts = [_prepare(c, dev) for c in clips]
    slots = []
    for c, mt in zip(clips, mts):
        F, V, H, W = c.vis.shape
        slots.append(dict(splats=mt.splats, bins=mt.bins, n=c.scene.n, cams=mt.cams_host,
                          disp=torch.as_tensor(c.disp).to(dev).contiguous(),
                          vis=torch.as_tensor(c.vis).to(dev).contiguous(),
                          acc=torch.zeros(F, V, c.scene.n, 16, device=dev),
                          t_final=torch.zeros(V, H, W, device=dev)))
    # an empty set rides along and is skipped
    empty = _prepare(synth.make_clip("small", frames=1, n=10, views=1, width=32, height=32, seed=45), dev)
    slots.insert(2, dict(splats=empty.splats, bins=empty.bins, n=0, cams=empty.cams_host,
                         disp=torch.zeros(1, 1, 32, 32, 2, device=dev), vis=None,
                         acc=torch.zeros(1, 1, 10, 16, device=dev)))
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    log(f"batch: {len(slots)} slots, frames {[c['frames'] for c in CLIPS]}")
    api.splat_accumulate_batch(slots, mts[0].params, stats=stats)
    torch.cuda.synchronize()
    assert float(slots[2]["acc"].abs().sum()) == 0.0
    del slots[2]
    # the same frames one launch each
    single = []
    single_stats = torch.zeros(4, dtype=torch.int64, device=dev)
    for c, mt, sl in zip(clips, mts, slots):
        accs = []
        for f in range(c.disp.shape[0]):
            acc = torch.zeros_like(sl["acc"][f])
            st = torch.zeros(4, dtype=torch.int64, device=dev)
            # with t_final every pixel is visited, as in the batch (which
            # asks for t_final), so the pair counts compare one to one
            api.splat_accumulate(mt.splats, mt.bins, c.scene.n, mt.cams_host, sl["disp"][f].contiguous(),
                                 sl["vis"][f].contiguous(), mt.params, acc,
                                 t_final=torch.zeros_like(sl["t_final"]), stats=st)
            if f == 0:
                single_stats += st
            accs.append(acc)
        single.append(torch.stack(accs))
    torch.cuda.synchronize()
    return clips, slots, single, stats.cpu().numpy(), single_stats.cpu().numpy()


def test_batch_matches_oracle_per_frame(batch):
    clips, slots, _, _, _ = batch
    for ci, (c, sl) in enumerate(zip(clips, slots)):
        geom = oracle.geometry(c.scene, c.cams)
        cov, conic = oracle.project64(c.scene, c.cams)
        lists = oracle.cell_lists(geom, c.cams, 1)
        acc = sl["acc"].cpu().numpy()
        for f in range(c.disp.shape[0]):
            comp = oracle.composite(c.scene, c.cams, geom, conic, lists, c.disp[f], c.vis[f])
            nbad, ntot, info = compare_accumulators(acc[f], comp)
            log(f"clip {ci} frame {f}: {nbad}/{ntot} outside tolerance, {info}")
            assert nbad == 0, info
            if f == 0:
                ok = comp["pixmarg"] == 0
                tf = sl["t_final"].cpu().numpy()
                np.testing.assert_allclose(tf[ok], comp["tfinal"][ok], rtol=1e-4, atol=1e-6)


def test_batch_equals_single_launches(batch):
    clips, slots, single, stats_b, stats_s = batch
    for c, sl, ref in zip(clips, slots, single):
        a = sl["acc"].cpu().double().numpy()
        b = ref.cpu().double().numpy()
        scale = np.abs(b).max(axis=(0, 1, 2), keepdims=True) + 1e-30
        assert np.all(np.abs(a - b) <= 1e-5 * scale + 1e-6 * np.abs(b)), np.abs(a - b).max()
    # frames share the evaluation: pair counts equal one frame per set
    assert stats_b[0] == stats_s[0] and stats_b[1] == stats_s[1], (stats_b, stats_s)
