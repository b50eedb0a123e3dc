"""Pin of the contributor order: vectorised tile lists == Python `sorted`."""

import numpy as np
import pytest

import scenes
from oracle import decide32, order


@pytest.mark.parametrize("cfg,v,tile", [(1, 0, 16), (1, 2, 8), (2, 12, 16), (2, 40, 32)])
def test_tile_lists_match_bruteforce(cfg, v, tile):
    c = scenes.make_config(cfg, scale_n=0.01 if cfg > 1 else 1.0)
    p = dict(c.params, tile=tile)
    d = decide32.project_cull32(c.scene, c.views.W[v], c.views.K[v], c.views.wh[v],
                                int(c.views.tstep[v]), p)
    ids = np.nonzero(d["surv"])[0]
    a = order.tile_lists(ids, d["depth_bits"], d["x0"], d["x1"], d["y0"], d["y1"], d["gx"], d["gy"])
    b = order.tile_lists_bruteforce(ids, d["depth_bits"], d["x0"], d["x1"], d["y0"], d["y1"],
                                    d["gx"], d["gy"])
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert a[1].size > 0


def test_ties_broken_by_id():
    db = np.array([7, 3, 7, 3, 1], np.uint32)
    np.testing.assert_array_equal(order.global_order(np.arange(5), db), [4, 1, 3, 0, 2])


def test_depth_bits_order_like_values():
    z = np.sort(np.random.default_rng(0).uniform(0.2, 3000, 1000).astype(np.float32))
    bits = z.view(np.uint32)
    assert np.all(np.diff(bits.astype(np.int64)) >= 0)
