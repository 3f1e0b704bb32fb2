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


# --- pins for the K-means start and the fraction-control ranking -----------------

def test_kmeans_initial_centres_hand_worked():
    """Hand-worked histograms whose final partition depends on the initial
    centres, the tie rule and the empty-cluster rule (traces in the fixture)."""
    g = json.load(open(os.path.join(GOLD, "kmeans_init_hand.json")))
    for case in g["cases"]:
        h = np.zeros(256, np.int64)
        for b, c in case["bins"].items():
            h[int(b)] = c
        bl, cS, cN, _ = oracle.kmeans_bins(h, case["K"])
        for b, lab in case["labels"].items():
            assert bl[int(b)] == lab, (case["bins"], b)
        assert np.all(bl[h == 0] == -1)
        for i, (s, n) in enumerate(case["centres"]):
            assert Fraction(int(cS[i]), int(cN[i])) == Fraction(s, n), (i, cS, cN)


_M64 = (1 << 64) - 1


def _splitmix64_mix(z):
    """SplitMix64's output function (Steele, Lea & Flood, OOPSLA 2014) on uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def test_splitmix64_published_vector():
    # The reference generator seeded with 1234567 (state += 0x9E3779B97F4A7C15,
    # then the output function) starts with these published values.
    s = 1234567
    expect = [6457827717110365317, 3203168211198807973, 9817491932198370423,
              4593380528125082431, 16408922859458223821]
    for e in expect:
        s = (s + 0x9E3779B97F4A7C15) & _M64
        assert int(_splitmix64_mix(np.uint64(s))) == e


def _ranked_selection(rmap, frac, seed):
    """The fraction-control ranking computed with library routines: border
    columns (class 0, by index); refined pixels (class 1) by 8-connected
    component size descending (scipy.ndimage.label), then index; the rest
    (class 2) by chessboard distance to classes 0 and 1
    (scipy.ndimage.distance_transform_cdt), then the hash of (index ^ seed),
    then index. The first round(frac * W * H), ascending."""
    H, W = rmap.shape
    N = W * H
    idx = np.arange(N, dtype=np.int64)
    border = np.zeros((H, W), bool)
    border[:, 0] = border[:, W - 1] = True
    refined = rmap.astype(bool)
    lab, _ = ndi.label(refined, structure=np.ones((3, 3)))
    sizes = np.bincount(lab.reshape(-1))
    dist = ndi.distance_transform_cdt(~(border | refined), metric="chessboard").reshape(-1)
    b = border.reshape(-1)
    r = refined.reshape(-1) & ~b
    cls = np.where(b, 0, np.where(r, 1, 2))
    prim = np.where(b, 0, np.where(r, -sizes[lab.reshape(-1)], dist)).astype(np.int64)
    hsh = _splitmix64_mix(idx.astype(np.uint64) ^ np.uint64(seed & _M64))
    sec = np.where(cls == 2, hsh, idx.astype(np.uint64))
    order = np.lexsort((idx, sec, prim, cls))
    want = min(N, int(round(frac * N)))
    return np.sort(order[:want]).astype(np.uint32), int(b.sum()), int(r.sum())


def _rect_scene(W, H, seed):
    """A piecewise-constant gray image: rectangles of distinct sizes and four
    well-separated levels, so the refined set has components of many sizes."""
    rng = np.random.default_rng(seed)
    img = np.full((H, W), 30, np.uint8)
    for k in range(14):
        w, h = int(rng.integers(6, W // 3)), int(rng.integers(6, H // 3))
        x, y = int(rng.integers(1, W - w - 1)), int(rng.integers(1, H - h - 1))
        img[y:y + h, x:x + w] = (90, 150, 220)[k % 3]
    return img


@pytest.mark.parametrize("case", ["rects", "tsukuba_gray"])
def test_fraction_control_ranking_matches_library_routines(case):
    if case == "rects":
        img = _rect_scene(160, 120, 11)
        seed = 0x1234
    else:
        spec = scenes.PRESETS[case]
        img = scenes.make_frame(spec).left
        seed = spec.seed
    H, W = img.shape[:2]
    N = W * H
    _, rmap = oracle.boundaries(img, K=4, mode=0, min_cc=50, return_map=True)
    _, nb, nr = _ranked_selection(rmap, 0.0, seed)
    assert nr > 200, "the map must hold refined pixels beyond the border columns"
    # cuts inside class 0, inside class 1 (component size order decides),
    # just past it and deep into class 2 (distance, then hash, decides)
    wants = [nb // 2, nb + nr // 3, nb + (2 * nr) // 3, nb + nr + 5, nb + nr + (N - nb - nr) // 4,
             nb + nr + (N - nb - nr) // 2, N]
    for want in wants:
        frac = want / N
        got = oracle.boundaries(img, K=4, mode=0, min_cc=50, frac=frac, seed=seed)
        exp, _, _ = _ranked_selection(rmap, frac, seed)
        np.testing.assert_array_equal(got, exp, err_msg=f"{case} want={want}")


def test_fraction_control_size_order_and_distance_decide():
    """On the rectangle scene the cut inside class 1 keeps whole large
    components before small ones, and the cut inside class 2 keeps every
    pixel at distance 1 before any pixel at distance 3."""
    img = _rect_scene(160, 120, 11)
    H, W = img.shape
    _, rmap = oracle.boundaries(img, K=4, mode=0, min_cc=50, return_map=True)
    lab, n = ndi.label(rmap.astype(bool), structure=np.ones((3, 3)))
    sizes = np.bincount(lab.reshape(-1))[1:]
    assert np.unique(sizes).size >= 3
    border = np.zeros((H, W), bool)
    border[:, 0] = border[:, W - 1] = True
    nb = int(border.sum())
    inner = rmap.astype(bool) & ~border
    biggest = np.argmax(sizes) + 1
    nbig = int((inner & (lab == biggest)).sum())
    got = oracle.boundaries(img, K=4, mode=0, min_cc=50, frac=(nb + nbig) / (W * H), seed=1)
    taken = np.zeros(W * H, bool)
    taken[got] = True
    np.testing.assert_array_equal(taken.reshape(H, W) & inner, inner & (lab == biggest))
    dist = ndi.distance_transform_cdt(~(border | rmap.astype(bool)), metric="chessboard")
    n1 = int((dist == 1).sum())
    got = oracle.boundaries(img, K=4, mode=0, min_cc=50, frac=(nb + int(inner.sum()) + n1) / (W * H), seed=1)
    taken = np.zeros(W * H, bool)
    taken[got] = True
    taken = taken.reshape(H, W)
    assert np.all(taken[dist == 1]) and not np.any(taken[dist >= 2])


@pytest.mark.parametrize("density,seed", [(0.002, 21), (0.01, 22), (0.05, 23)])
def test_fraction_select_on_sparse_maps_matches_library_routines(density, seed):
    """Fraction control on arbitrary refined maps: isolated pixels and short
    runs, where every term of the chessboard distance and every component
    size matter, against the ranking built from scipy routines."""
    rng = np.random.default_rng(seed)
    H, W = 57, 83
    rmap = (rng.random((H, W)) < density).astype(np.uint8)
    for _ in range(6):   # a few short horizontal and vertical runs of various lengths
        y, x, L = int(rng.integers(0, H)), int(rng.integers(0, W - 9)), int(rng.integers(2, 9))
        if rng.random() < 0.5:
            rmap[y, x:x + L] = 1
        else:
            rmap[max(0, y - L):y, x] = 1
    _, nb, nr = _ranked_selection(rmap, 0.0, seed)
    N = W * H
    natural = oracle.fraction_select(rmap, -1.0)
    border = np.zeros((H, W), bool)
    border[:, 0] = border[:, W - 1] = True
    np.testing.assert_array_equal(natural, np.flatnonzero(border | rmap.astype(bool)).astype(np.uint32))
    for want in sorted({nb // 3, nb + nr // 2, nb + nr + 1, nb + nr + (N - nb - nr) // 8,
                        nb + nr + (N - nb - nr) // 3, nb + nr + (2 * (N - nb - nr)) // 3, N}):
        got = oracle.fraction_select(rmap, want / N, seed)
        exp, _, _ = _ranked_selection(rmap, want / N, seed)
        assert got.size == want
        np.testing.assert_array_equal(got, exp, err_msg=f"want={want}")
