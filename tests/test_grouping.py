"""The test-side transform from the oracle's per-tile lists to the library's
4x4-tile-group layout (CPU): both constructions agree bit for bit, and the
grouped runs expand back to exactly the per-tile lists."""
import numpy as np
import pytest

import oracle
from paper_2501_08174_amd import scenes
from tests.grouping import (expand_to_tile_lists, grouped_from_rectangles, grouped_from_tile_lists,
                            instance_count)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_grouped_layout_from_tile_lists(tile):
    """Every tile's entries of its group run (sub-rectangle contains the
    tile) are exactly its per-tile list, in the same order; each (group,
    surfel) pair appears once, when the surfel's tile rectangle meets the
    group; the list-derived and rectangle-derived layouts are identical."""
    rp = oracle.RasterParams(tile_w=tile[0], tile_h=tile[1])
    sc = scenes.make_random_scene(16, 300, n_views=3, width=[140, 61, 17], height=[97, 130, 33],
                                  scale_range=(0.02, 0.6))
    geoms = [oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, c, rp) for c in sc.cams]
    k1, v1, r1 = oracle.bin64(geoms, sc.cams, rp)
    k4, v4, r4 = grouped_from_tile_lists(k1, v1, r1, sc.cams, *tile)
    kd, vd, rd = grouped_from_rectangles(geoms, sc.cams, *tile)
    np.testing.assert_array_equal(k4, kd)
    np.testing.assert_array_equal(v4, vd)
    np.testing.assert_array_equal(r4, rd)
    ids, rg = expand_to_tile_lists(v4, r4, sc.cams, *tile)
    np.testing.assert_array_equal(ids, v1)
    np.testing.assert_array_equal(rg, r1)
    assert k4.size == instance_count(geoms) < k1.size
    gk = (k4 >> np.uint64(32)).astype(np.int64)
    pair = gk * (sc.n + 1) + (v4 & np.uint32(0xFFFFFF)).astype(np.int64)
    assert np.unique(pair).size == pair.size
    assert np.all(np.diff(gk) >= 0)
    # large rectangles span several groups, small ones one
    sub = v4 >> np.uint32(24)
    spans = ((sub >> 2) & 3) - (sub & 3) + 1
    assert (spans == 4).any() and (spans == 1).any()
