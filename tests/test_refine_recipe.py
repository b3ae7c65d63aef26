"""Host logic of the 3DGS refinement recipe (Sec. 4.6 refines as 3DGS does):
the per-parameter learning rates, the exponential position-rate decay and the
scene-extent scale.  No GPU."""
import math

import numpy as np
import pytest

import synth
from paper_2604_02586_amd import _lib
from paper_2604_02586_amd.raster import LR_3DGS, lr_3dgs, scene_extent


def test_scene_extent_of_known_centres():
    # four cameras on a circle of radius 3 around (1, 2, 0): the centres'
    # mean is (1, 2, 0) and every centre is 3 from it
    cams = [synth.look_at_camera((1 + 3 * math.cos(a), 2 + 3 * math.sin(a), 0.0), (1, 2, 0), (0, 0, 1), 64, 48, 60)
            for a in np.linspace(0, 2 * math.pi, 4, endpoint=False)]
    assert scene_extent(_lib.cameras(cams)) == pytest.approx(3.3, rel=1e-5)
    # one camera off the circle sets the extent
    cams.append(synth.look_at_camera((1, 2, 10.0), (1, 2, 0), (0, 1, 0), 64, 48, 60))
    mean = np.array([1, 2, 2.0])
    far = max(np.linalg.norm(np.array(c) - mean) for c in
              [(1 + 3 * math.cos(a), 2 + 3 * math.sin(a), 0.0) for a in np.linspace(0, 2 * math.pi, 4,
                                                                                        endpoint=False)]
              + [(1, 2, 10.0)])
    assert scene_extent(_lib.cameras(cams)) == pytest.approx(1.1 * far, rel=1e-5)


def test_rates_and_decay():
    K = 16
    lr0 = lr_3dgs(0, 2.0, K)
    assert lr0[0] == pytest.approx(1.6e-4 * 2.0)
    assert lr0[1:4] == [1e-3, 5e-3, 0.05]
    assert lr0[4] == (2.5e-3, 2.5e-3 / 20, 3 * K, 3)
    # exponential (log-linear) decay: the midpoint is the geometric mean, the
    # end is the final rate, and the rate holds there afterwards
    steps = LR_3DGS["position_max_steps"]
    mid = lr_3dgs(steps // 2, 1.0, K)[0]
    assert mid == pytest.approx(math.sqrt(1.6e-4 * 1.6e-6), rel=1e-9)
    assert lr_3dgs(steps, 1.0, K)[0] == pytest.approx(1.6e-6, rel=1e-9)
    assert lr_3dgs(2 * steps, 1.0, K)[0] == pytest.approx(1.6e-6, rel=1e-9)
    # 1000 refinement iterations cover the first 1/30 of the schedule
    assert lr_3dgs(1000, 1.0, K)[0] == pytest.approx(1.6e-4 * 0.01 ** (1000 / 30000), rel=1e-9)
