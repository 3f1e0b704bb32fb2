"""Checks of the synthetic scene generator (input recipe, not the method)."""
import numpy as np
import pytest

import scenes


@pytest.mark.parametrize("name", ["tsukuba_gray", "serve_vga", "tsukuba_paper"])
def test_unoccluded_pixels_match_across_views(name):
    spec = scenes.PRESETS[name]
    f = scenes.make_frame(spec)
    H, W = f.gt.shape
    ys, xs = np.nonzero(f.occ == 0)
    xr = xs - f.gt[ys, xs].astype(int)
    assert np.all(xr >= 0)
    np.testing.assert_array_equal(f.left[ys, xs], f.right[ys, xr])
    assert f.gt.max() <= spec.dmax_regions


def test_deterministic_and_seed_sensitive():
    spec = scenes.PRESETS["tsukuba_gray"]
    a = scenes.make_frame(spec)
    b = scenes.make_frame(spec)
    c = scenes.make_frame(scenes.scaled(spec, seed=999))
    assert np.array_equal(a.left, b.left) and np.array_equal(a.right, b.right)
    assert not np.array_equal(a.left, c.left)


def test_contour_list_properties():
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    lst = scenes.contour_list(f.rid, 0.18, 1)
    assert lst.size == round(0.18 * spec.W * spec.H)
    assert np.all(np.diff(lst.astype(np.int64)) > 0)
    xs = lst % spec.W
    assert (xs == 0).sum() == spec.H and (xs == spec.W - 1).sum() == spec.H


def test_video_frames_match_single_frames():
    spec = scenes.scaled(scenes.PRESETS["uhd_video"], W=400, H=240, n_regions=8)
    fr = scenes.video_fracs(spec, 0, 3)
    left, right, lists = scenes.make_video(spec, 0, 3, fr)
    for t in range(3):
        f = scenes.make_frame(spec, t)
        assert np.array_equal(left[t], f.left) and np.array_equal(right[t], f.right)
        assert np.array_equal(lists[t], scenes.contour_list(f.rid, fr[t], spec.seed ^ t))
    assert not np.array_equal(left[0], left[2])
