"""Pins of the plain-C occlusion statistics (oracle/prune_native.c): the
hand-computed stacks of tests/golden/prune_stack.json, the vectorised torch
oracle's statistics on random multi-view scenes (an independent
implementation of the same per-pixel loop), and the hidden-surfel case of
Section 4.3 (CPU)."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle.prune_native import prune_stats_view64, prune_stats_views64
from oracle.render import TIE_KINDS, Params64, render_view
from paper_2501_08174_amd import scenes
from tests.oracle_scenes import front_camera, scene_from

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ID = [1.0, 0.0, 0.0, 0.0]


def test_hand_computed_stacks(rp):
    gold = json.load(open(os.path.join(GOLDEN, "prune_stack.json")))
    cam = front_camera(9)
    for case in gold["scenes"]:
        n = len(case["opacity"])
        sc = scene_from([[0.0, 0.0, z] for z in case["world_z"]], [(0.05, 0.05)] * n, [ID] * n, case["opacity"],
                        [(0.5, 0.5, 0.5)] * n, [cam])
        st = prune_stats_views64(sc.means, sc.scales, sc.quats, sc.opac, sc.cams, rp)
        np.testing.assert_array_equal(st["hits"], case["hits"], err_msg=case["name"])
        np.testing.assert_allclose(st["max_alpha"], case["max_alpha"], rtol=0, atol=1e-12, err_msg=case["name"])
        np.testing.assert_allclose(st["max_weight"], case["max_weight"], rtol=0, atol=1e-12, err_msg=case["name"])
        assert not st["prune"].any() and st["in_frustum"].all()


def _exposure_counts(res, n):
    """From the torch oracle's per-pixel decisions: for every pixel with a
    cutoff or termination tie entry, each entry from the first tie on that
    passes the cutoff up to the stop, each tie entry itself, and the next m
    entries past the stop that pass the cutoff (m the pixel's tie entries)
    count one for their surfel."""
    codes = [TIE_KINDS.index("cut"), TIE_KINDS.index("term")]
    tl = res["tie_list"]
    tl = tl[np.isin(tl[:, 2], codes)]
    out = np.zeros(n, np.int64)
    row0 = 0
    for d in res["decisions"]:
        P, L = d["gid"].shape
        for r in range(P):
            ent = tl[tl[:, 0] == row0 + r]
            if ent.size == 0:
                continue
            gids = d["gid"][r]
            cols = [int(np.nonzero(gids == gg)[0][0]) for gg in np.unique(ent[:, 1])]
            first, stop, m = min(cols), int(d["first_stop"][r]), len(cols)
            for c in range(first, min(stop, L - 1) + 1):
                if not d["skip"][r, c] or c in cols:
                    out[gids[c]] += 1
            c = stop + 1
            while m > 0 and c < L:
                if not d["skip"][r, c]:
                    out[gids[c]] += 1
                    m -= 1
                c += 1
        row0 += P
    return out


@pytest.mark.parametrize("seed", [71, 72])
def test_matches_torch_oracle_on_random_views(rp, seed, monkeypatch):
    """Every surfel's hits, maxima and tie exposure count (cutoff and
    termination ties and the decisions after them) equal those computed from
    render_pixels' decisions + prune_stats64 over whole views; the tie
    windows are widened (both oracles read the same ones) so that these
    scenes have ties."""
    import oracle.render as orr
    monkeypatch.setattr(orr, "TIE_CUTOFF_REL", 2e-2)
    monkeypatch.setattr(orr, "TIE_TERM_REL", 5e-2)
    sc = scenes.make_random_scene(seed, 400, n_views=3, width=[48, 37, 64], height=[40, 51, 30],
                                  scale_range=(0.01, 0.4))
    P = Params64.from_arrays(sc.means, sc.scales, sc.quats, sc.opac, sc.sh, sc.sh_degree)
    pairs, culled, tie = [], [], np.zeros(sc.n, np.int64)
    for cam in sc.cams:
        g = oracle.view_geometry64(sc.means, sc.scales, sc.quats, sc.opac, cam, rp)
        res, _ = render_view(P, cam, g, rp, keep_decisions=True)
        pairs.append(res["pairs"])
        culled.append(g["culled"])
        tie += _exposure_counts(res, sc.n)
    ref = oracle.prune_stats64(sc.n, pairs, culled)
    st = prune_stats_views64(sc.means, sc.scales, sc.quats, sc.opac, sc.cams, rp, workers=2)
    np.testing.assert_array_equal(st["hits"], ref["hits"])
    np.testing.assert_allclose(st["max_alpha"], ref["max_alpha"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(st["max_weight"], ref["max_weight"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(st["in_frustum"], ref["in_frustum"])
    np.testing.assert_array_equal(st["prune"], ref["prune"])
    np.testing.assert_array_equal(st["tie"], tie)
    assert (st["hits"] > 0).sum() > 100 and tie.sum() > 0


def test_hidden_surfel_in_frustum_is_pruned(rp):
    """A small surfel behind three opaque full-cover layers is inside the
    frustum but never blended (Section 4.3's case); one behind the camera
    and one below the cutoff opacity are neither."""
    cam = front_camera(40)
    means = [[0, 0, 0.0], [0, 0, 0.05], [0, 0, 0.1], [0, 0, 0.5], [0, 0, -5.0], [0.2, 0.1, -0.5]]
    sc = scene_from(means, [(5, 5)] * 3 + [(0.2, 0.2)] * 3, [ID] * 6, [0.99, 0.99, 0.99, 0.9, 0.9, 0.002],
                    [(1, 1, 1)] * 6, [cam])
    st = prune_stats_views64(sc.means, sc.scales, sc.quats, sc.opac, sc.cams, rp)
    assert list(st["in_frustum"]) == [True, True, True, True, False, False]
    assert (st["hits"][:3] > 0).all() and (st["hits"][3:] == 0).all()
    assert list(st["prune"]) == [False, False, False, True, True, True]
    # a pixel mask restricts the pixels rendered
    m = np.zeros((40, 40), np.uint8)
    m[5, 5] = 1         # T = 1, 0.07, 0.005 before the three layers: all blend
    one = prune_stats_view64(sc.means, sc.scales, sc.quats, sc.opac, cam, rp, pix_mask=m)
    assert list(one["hits"][:4]) == [1, 1, 1, 0]
