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
