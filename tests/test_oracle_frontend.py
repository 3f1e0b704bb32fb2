"""Pins for the oracle's segmentation front end (Sec. III: colour space
conversion, histogram K-means, boundary detection, refinement, connected
components) and the benchmark's fraction control.

Checks come from published values, library routines (scipy.ndimage) and
brute force over pixels, never from the oracle itself.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage as ndi

import oracle
import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --- lightness -----------------------------------------------------------------

def test_lightness_published_values():
    # CIE L* of sRGB black/white/mid-gray and primaries (standard published values):
    # black 0, white 100, sRGB gray 119 -> L* 50.0, red 53.24, green 87.73, blue 32.30.
    px = np.array([[[0, 0, 0], [255, 255, 255], [119, 119, 119], [255, 0, 0], [0, 255, 0], [0, 0, 255]]], np.uint8)
    L = oracle.lightness(px)[0]
    expect = [0.0, 100.0, 50.0, 53.24, 87.73, 32.30]
    for got, ls in zip(L, expect):
        assert abs(int(got) - ls * 2.55) <= 0.75, (got, ls)
    assert L[0] == 0 and L[1] == 255


def test_lightness_monotone_on_gray_ramp_and_gray_passthrough():
    ramp = np.repeat(np.arange(256, dtype=np.uint8)[None, :, None], 3, 2)
    L = oracle.lightness(ramp)[0].astype(int)
    assert np.all(np.diff(L) >= 0)
    g = np.arange(256, dtype=np.uint8).reshape(16, 16)
    np.testing.assert_array_equal(oracle.lightness(g), g)


def test_histogram_counts_every_pixel():
    img = np.random.default_rng(0).integers(0, 256, (37, 51), dtype=np.uint8)
    h = oracle.histogram(img)
    assert h.sum() == img.size
    np.testing.assert_array_equal(h, np.bincount(img.reshape(-1), minlength=256))


# --- K-means on histogram bins ---------------------------------------------------

def _pixel_kmeans(vals, K):
    """Lloyd's algorithm run on the pixels themselves (not the bins), exact rationals."""
    lo, hi = int(vals.min()), int(vals.max())
    cent = [Fraction(lo + ((2 * k + 1) * (hi - lo + 1)) // (2 * K)) for k in range(K)]
    assign = None
    for _ in range(1000):
        new = []
        for v in vals:
            dist = [abs(Fraction(int(v)) - c) for c in cent]
            new.append(min(range(K), key=lambda k: (dist[k], k)))   # ties to the lower k
        if new == assign:
            break
        assign = new
        for k in range(K):
            members = [int(v) for v, a in zip(vals, assign) if a == k]
            if members:
                cent[k] = Fraction(sum(members), len(members))
    order = sorted(range(K), key=lambda k: (cent[k], k))
    rank = {k: i for i, k in enumerate(order)}
    return np.array([rank[a] for a in assign]), [cent[k] for k in order]


@pytest.mark.parametrize("K,seed", [(2, 0), (3, 1), (4, 2), (5, 3)])
def test_bin_kmeans_equals_pixel_kmeans(K, seed):
    rng = np.random.default_rng(seed)
    # a mixture of a few lightness modes, small enough for pixel-wise Lloyd in Python
    modes = rng.integers(20, 235, K)
    vals = np.clip(rng.normal(modes[rng.integers(0, K, 300)], 12), 0, 255).astype(np.uint8)
    h = oracle.histogram(vals)
    bl, cS, cN, _ = oracle.kmeans_bins(h, K)
    got = oracle.label_pixels(vals, bl)
    exp, cents = _pixel_kmeans(vals, K)
    np.testing.assert_array_equal(got, exp)
    for i in range(K):
        if cN[i] > 0:
            assert Fraction(int(cS[i]), int(cN[i])) == cents[i]


def test_kmeans_one_cluster_and_two_levels():
    img = np.random.default_rng(1).integers(0, 256, 500, dtype=np.uint8)
    bl, *_ = oracle.kmeans_bins(oracle.histogram(img), 1)
    assert np.all(oracle.label_pixels(img, bl) == 0)
    two = np.array([40] * 100 + [200] * 50, np.uint8)
    bl, cS, cN, _ = oracle.kmeans_bins(oracle.histogram(two), 2)
    lab = oracle.label_pixels(two, bl)
    assert np.all(lab[:100] == 0) and np.all(lab[100:] == 1)
    assert cS[0] / cN[0] == 40 and cS[1] / cN[1] == 200


# --- morphology, boundary, refinement --------------------------------------------

def test_erode_dilate_match_scipy():
    lab = np.random.default_rng(2).integers(0, 4, (31, 45), dtype=np.uint8)
    np.testing.assert_array_equal(oracle.erode3(lab), ndi.grey_erosion(lab, size=3, mode="nearest"))
    np.testing.assert_array_equal(oracle.dilate3(lab), ndi.grey_dilation(lab, size=3, mode="nearest"))


def test_open_close_matches_scipy_and_is_idempotent():
    lab = np.random.default_rng(3).integers(0, 4, (40, 52), dtype=np.uint8)
    got = oracle.label_open_close(lab)
    o = ndi.grey_dilation(ndi.grey_erosion(lab, size=3, mode="nearest"), size=3, mode="nearest")
    exp = ndi.grey_erosion(ndi.grey_dilation(o, size=3, mode="nearest"), size=3, mode="nearest")
    np.testing.assert_array_equal(got, exp)
    # opening is idempotent
    op = lambda m: oracle.dilate3(oracle.erode3(m))
    np.testing.assert_array_equal(op(op(lab)), op(lab))
    speck = np.zeros((9, 9), np.uint8); speck[4, 4] = 3
    assert oracle.label_open_close(speck).max() == 0


def test_boundary_is_moore_neighbour_difference():
    lab = np.random.default_rng(4).integers(0, 3, (29, 41), dtype=np.uint8)
    exp = (ndi.maximum_filter(lab, 3, mode="nearest") != ndi.minimum_filter(lab, 3, mode="nearest")).astype(np.uint8)
    np.testing.assert_array_equal(oracle.boundary(lab), exp)
    step = np.zeros((6, 10), np.uint8); step[:, 6:] = 1
    B = oracle.boundary(step)
    assert set(np.flatnonzero(B.any(0))) == {5, 6}


def test_fill_worked_example_from_paper():
    g = json.load(open(os.path.join(GOLD, "fill_paper_example.json")))
    B = np.array(g["input"], np.uint8)
    big = np.zeros((5, 5), np.uint8); big[1:4, 1:4] = B
    F = oracle.fill(big)
    assert F[2, 2] == g["centre_after_fill"]
    Rm = oracle.remove(F)
    np.testing.assert_array_equal(Rm[1:4, 1:4], np.array(g["after_fill_then_remove"], np.uint8))


def test_fill_remove_match_neighbour_counts():
    B = (np.random.default_rng(5).random((33, 47)) < 0.7).astype(np.uint8)
    k8 = np.ones((3, 3), int); k8[1, 1] = 0
    n8 = ndi.convolve(B.astype(int), k8, mode="constant", cval=0)
    np.testing.assert_array_equal(oracle.fill(B), (B | (n8 == 8)).astype(np.uint8))
    k4 = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]])
    n4 = ndi.convolve(B.astype(int), k4, mode="constant", cval=0)
    np.testing.assert_array_equal(oracle.remove(B), (B & ~(n4 == 4)).astype(np.uint8))


def test_components_match_scipy_label():
    B = (np.random.default_rng(6).random((60, 70)) < 0.45).astype(np.uint8)
    comp, sizes = oracle.components(B)
    lab, n = ndi.label(B, structure=np.ones((3, 3)))
    assert len(sizes) == n
    np.testing.assert_array_equal(np.sort(sizes), np.sort(np.bincount(lab.reshape(-1))[1:]))
    # same partition: each oracle component maps to exactly one scipy component
    m = B.astype(bool)
    pairs = set(zip(comp[m].tolist(), lab[m].tolist()))
    assert len(pairs) == n


def test_cc_filter_min_size_and_four_percent_rule():
    B = (np.random.default_rng(7).random((80, 90)) < 0.42).astype(np.uint8)
    K = oracle.cc_filter(B, mode=0, min_size=50)
    lab, n = ndi.label(B, structure=np.ones((3, 3)))
    sizes = np.bincount(lab.reshape(-1))
    keep = np.isin(lab, np.flatnonzero(sizes >= 50)) & (lab > 0)
    np.testing.assert_array_equal(K, keep.astype(np.uint8))
    # 4% rule on a constructed map: component sizes 1, 2, 3 and 100 (total 106, 4% = 4.24):
    # 1 and 2 go (3 <= 4.24), adding 3 would make 6 > 4.24.
    M = np.zeros((20, 40), np.uint8)
    M[0, 0] = 1
    M[0, 5:7] = 1
    M[0, 10:13] = 1
    M[5:15, 20:30] = 1
    out = oracle.cc_filter(M, mode=1, drop_frac=0.04)
    assert out[0, 0] == 0 and out[0, 5:7].sum() == 0 and out[0, 10:13].sum() == 3 and out[5:15, 20:30].sum() == 100


# --- full front end + fraction control --------------------------------------------

@pytest.mark.parametrize("name", ["tsukuba_gray", "serve_vga"])
def test_frontend_list_properties(name):
    spec = scenes.PRESETS[name]
    f = scenes.make_frame(spec)
    natural, rmap = oracle.boundaries(f.left, K=4, mode=0, min_cc=50, return_map=True)
    W, H = spec.W, spec.H
    assert np.all(np.diff(natural.astype(np.int64)) > 0)
    xs = natural % W
    # every row holds its two border pixels (Sec. III: map borders count as boundary)
    assert np.array_equal(np.bincount((natural[xs == 0] // W).astype(int), minlength=H), np.ones(H))
    assert np.array_equal(np.bincount((natural[xs == W - 1] // W).astype(int), minlength=H), np.ones(H))
    # refined map has no component smaller than 50
    _, sizes = oracle.components(rmap)
    assert sizes.size == 0 or sizes.min() >= 50
    fr = []
    for frac in (0.12, 0.18, 0.24):
        lst = oracle.boundaries(f.left, K=4, mode=0, min_cc=50, frac=frac, seed=spec.seed)
        assert lst.size == round(frac * W * H)
        assert np.all(np.diff(lst.astype(np.int64)) > 0)
        fr.append(lst)
    assert np.all(np.isin(fr[0], fr[1])) and np.all(np.isin(fr[1], fr[2]))   # prefix property


def test_paper_mode_frontend_runs():
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    lst = oracle.boundaries(f.left, K=10, mode=1)
    assert lst.size >= 2 * spec.H and np.all(np.diff(lst.astype(np.int64)) > 0)
