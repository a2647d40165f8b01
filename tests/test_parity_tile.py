"""The sampled-tile oracle used at full size (CPU): on a tile that a few
windows overlap, the object gradient summed over those windows on a crop of
the object equals the full oracle's object gradient there."""
import numpy as np

import synth
from tests import parity_util as U


def test_cropped_tile_equals_the_full_oracle():
    case = U.make_case(synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                                     mode_weights=(0.75, 0.25), K=40, name="C1-tile"),
                       with_sigma=True, with_bg=True, with_mask=True, pads=(80, 64))
    w = case["w"]
    ty, tx, hit = U.sparse_object_tile(case["pos"], w.N, w.H, w.W, th=16, tw=64, lo=2, hi=5)
    assert 2 <= len(hit) <= 5
    full = U.oracle_grads(case, kind=1)["g_object"][..., ty:ty + 16, tx:tx + 64]
    tile = U.oracle_object_tile(case, ty, tx, hit, kind=1)
    assert np.abs(full).max() > 0
    np.testing.assert_allclose(tile, full, rtol=0, atol=1e-12 * np.abs(full).max())
