"""GPU parity of the motion-transfer path (HIP via the C ABI) against the
CPU oracle, stage by stage and end to end, on seeded synthetic inputs."""
import numpy as np
import pytest

import oracle
import synth
from helpers import (check_accumulate, check_bins, check_end_to_end, check_preprocess, check_solve, dump, log,
                     oracle_full, run_gpu)

pytestmark = pytest.mark.gpu

# small sizes that still span several tiles and coarse bins plus a ragged tail
CASES = {
    "small": dict(name="small"),                                     # 2k G, 4 views, 128x128
    "ragged": dict(name="small", seed=7, n=3000, views=3, width=333, height=250),
    "medium_lite": dict(name="medium", seed=5, n=20000, views=5, width=420, height=300),
}


def _workload(case):
    kw = dict(CASES[case])
    return synth.make_workload(kw.pop("name"), **kw)


@pytest.fixture(scope="module", params=list(CASES))
def pair(request):
    log(f"[case {request.param}] generating")
    wl = _workload(request.param)
    log(f"[case {request.param}] oracle")
    ref = oracle_full(wl)
    log(f"[case {request.param}] gpu")
    gpu = run_gpu(wl)
    dump(request.param, gpu)
    log(f"[case {request.param}] ready")
    return request.param, wl, ref, gpu


def test_preprocess_parity(pair):
    check_preprocess(*pair)


def test_bin_sort_bit_exact(pair):
    check_bins(*pair)


def test_accumulate_parity(pair):
    check_accumulate(*pair)


def test_solve_views_parity(pair):
    check_solve(*pair)


def test_end_to_end_parity(pair):
    check_end_to_end(*pair)



@pytest.mark.parametrize("records", [0, 1001, 3_000_000])
def test_acc_zero_clears_every_record(records):
    import torch
    from paper_2604_02586_amd import api
    log(f"[acc_zero records={records}]")
    a = torch.full((records + 1, 16), float("nan"), dtype=torch.float32, device="cuda:0")
    api.acc_zero(a[:records])
    torch.cuda.synchronize()
    assert int(torch.count_nonzero(a[:records].view(torch.int32)).item()) == 0
    assert bool(torch.isnan(a[records]).all())      # the record past the end is untouched


def test_hidden_track_pixels_skipped_without_t_final():
    """Without t_final, pixels whose track is hidden are never visited: the
    accumulators are the same (up to the order of the FP32 atomics) and the
    counters drop by those pixels' work."""
    import torch
    from paper_2604_02586_amd import api
    dev = torch.device("cuda:0")
    log("[hidden-track pixels]")
    wl = _workload("ragged")
    vis = (np.random.default_rng(3).random(np.asarray(wl.vis).shape) < 0.9).astype(np.uint8)
    hidden = float((vis == 0).mean())
    assert hidden > 0.05, hidden
    g = api.GaussianTensors.from_scene(wl.scene, dev)
    mt = api.MotionTransfer(wl.cams, wl.scene.n, dev)
    d = torch.as_tensor(wl.disp).to(dev).contiguous()
    vv = torch.as_tensor(vis).to(dev).contiguous()
    mt.preprocess(g)
    mt.bin_sort()
    mt.accumulate(d, vv, t_final=True, stats=True)
    torch.cuda.synchronize()
    acc_t, st_t = mt.acc.cpu().numpy(), mt.stats.cpu().numpy().copy()
    mt.accumulate(d, vv, t_final=False, stats=True)
    torch.cuda.synchronize()
    acc_n, st_n = mt.acc.cpu().numpy(), mt.stats.cpu().numpy().copy()
    scale = np.abs(acc_t).max(axis=(0, 1)) + 1e-30
    assert (np.abs(acc_n - acc_t) <= 1e-5 * scale).all()
    log(f"  hidden {hidden:.3f}; evaluated {st_t[0]} -> {st_n[0]}, pixel steps {st_t[2]} -> {st_n[2]}")
    assert st_n[0] < st_t[0] and st_n[1] < st_t[1] and st_n[2] < st_t[2]
    # with every track visible, every pixel is visited again: the same walk
    # as with t_final (termination does not depend on visibility)
    mt.accumulate(d, None, t_final=False, stats=True)
    torch.cuda.synchronize()
    st_a = mt.stats.cpu().numpy()
    assert st_a[0] == st_t[0] and st_a[1] == st_t[1] and st_a[2] == st_t[2], (st_a, st_t)
