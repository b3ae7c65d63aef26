"""GPU parity at the benchmark's full shapes, whole frame, in the launch
configuration the benchmark times (no per-pixel transmittance output, no
pair counters): 1M Gaussians x 20 views x 1920x1080 with large motions, 5%
outlier tracks and 0.9 visibility, and 300k Gaussians x 27 views x
1352x1014.  Every stage against the oracle on every Gaussian and view
(the expanded per-tile lists are compared at the small sizes only; the
coarse lists they are filtered from are compared here)."""
import time

import pytest

import synth
from helpers import (check_accumulate, check_bins, check_end_to_end, check_preprocess, check_solve, log,
                     oracle_full, run_gpu)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", params=["medium", "large"])
def full(request):
    t0 = time.perf_counter()
    log(f"[full {request.param}] generating")
    wl = synth.make_workload(request.param)
    log(f"[full {request.param}] {wl.scene.n} Gaussians x {len(wl.cams)} views x {wl.cams[0].W}x{wl.cams[0].H}; "
        f"gpu (benchmark launch configuration)")
    gpu = run_gpu(wl, t_final=False, stats=False)
    log(f"[full {request.param}] oracle ({time.perf_counter() - t0:.0f} s so far)")
    ref = oracle_full(wl)
    log(f"[full {request.param}] ready after {time.perf_counter() - t0:.0f} s")
    yield request.param, wl, ref, gpu
    del gpu, ref


@pytest.mark.timeout(1200)
def test_full_preprocess_and_bins(full):
    check_preprocess(*full)
    check_bins(*full, expand=False)


@pytest.mark.timeout(1200)
def test_full_accumulate(full):
    check_accumulate(*full)


@pytest.mark.timeout(1200)
def test_full_solve_views(full):
    check_solve(*full)


@pytest.mark.timeout(1200)
def test_full_end_to_end(full):
    check_end_to_end(*full)
