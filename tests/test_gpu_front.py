"""GPU parity of the front end (lightness -> histogram K-means -> labels ->
refinement -> components -> filter -> list) against the oracle, bit-exact:
the list, the kept boundary map and the label image."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def sbs():
    import paper_2001_07809_amd as m
    m.lib()
    return m


def oracle_labels(img, K, mode):
    L8 = oracle.lightness(img)
    bl, _, _, _ = oracle.kmeans_bins(oracle.histogram(L8), K)
    lab = oracle.label_pixels(L8, bl)
    return oracle.label_open_close(lab) if mode == 0 else lab


def check(torch, sbs, img, K, mode, min_cc=50, what=""):
    d = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    lst, refined, labels = sbs.boundaries(d, K=K, mode=mode, min_cc=min_cc, with_maps=True)
    exp_list, exp_map = oracle.boundaries(img, K=K, mode=mode, min_cc=min_cc, frac=-1.0, return_map=True)
    exp_lab = oracle_labels(img, K, mode)
    got_lab = labels.cpu().numpy()
    assert np.array_equal(got_lab, exp_lab), f"{what}: labels differ at {np.argwhere(got_lab != exp_lab)[:5]}"
    got_map = refined.cpu().numpy()
    assert np.array_equal(got_map, exp_map), f"{what}: refined map differs at {np.argwhere(got_map != exp_map)[:5]}"
    got = lst.cpu().numpy().view(np.uint32)
    assert got.size == exp_list.size and np.array_equal(got, exp_list), f"{what}: list differs"
    return got


def test_lightness_exhaustive_over_all_rgb_colours(torch, sbs):
    i = np.arange(1 << 24, dtype=np.uint32)
    img = np.stack([(i & 255), (i >> 8) & 255, i >> 16], -1).astype(np.uint8).reshape(4096, 4096, 3)
    got = sbs.lightness(torch.from_numpy(img).cuda()).cpu().numpy()
    exp = oracle.lightness(img)
    bad = np.flatnonzero(got != exp)
    assert bad.size == 0, f"{bad.size} colours differ, first {img.reshape(-1, 3)[bad[:5]]}: {got.ravel()[bad[:5]]} vs {exp.ravel()[bad[:5]]}"
    gray = np.arange(256, dtype=np.uint8).reshape(16, 16)
    assert np.array_equal(sbs.lightness(torch.from_numpy(gray).cuda()).cpu().numpy(), gray)


@pytest.mark.parametrize("name", ["tsukuba_gray", "middlebury_rgb"])
@pytest.mark.parametrize("mode,K", [(0, 4), (1, 10)])
def test_front_end_on_scenes(torch, sbs, name, mode, K):
    f = scenes.make_frame(scenes.PRESETS[name])
    got = check(torch, sbs, f.left, K, mode, what=f"{name} mode {mode}")
    assert got.size > 0


def test_front_end_noise_many_components(torch, sbs):
    """Noise gives thousands of small components with equal sizes: the 4% rule's
    tie order (raster order of each component's first pixel) and union-find
    under contention."""
    rng = np.random.default_rng(3)
    for (H, W, C) in [(300, 410, 3), (512, 512, 1), (97, 1203, 1)]:
        shape = (H, W, C) if C == 3 else (H, W)
        img = rng.integers(0, 256, shape, dtype=np.uint8)
        img = (img // 128 * 255).astype(np.uint8) if C == 1 else img
        for mode, K in [(0, 2), (1, 2), (1, 6)]:
            check(torch, sbs, img, K, mode, what=f"noise {shape} mode {mode} K {K}")
    # sparse dots: isolated single pixels in paper mode (all components of size 8/9)
    img = np.zeros((200, 300), np.uint8)
    img[5::7, 3::11] = 200
    check(torch, sbs, img, 2, 1, what="dots paper")
    check(torch, sbs, img, 2, 0, min_cc=0, what="dots configured min_cc 0")


def test_front_end_degenerate_shapes(torch, sbs):
    rng = np.random.default_rng(4)
    for (H, W) in [(1, 1), (1, 37), (41, 1), (2, 2), (3, 5)]:
        img = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        for mode in (0, 1):
            for K in (1, 3, 64):
                check(torch, sbs, img, K, mode, min_cc=1, what=f"{H}x{W} mode {mode} K {K}")
    const = np.full((60, 70), 90, np.uint8)
    lst = check(torch, sbs, const, 5, 0, what="constant")
    assert lst.size == 2 * 60   # border columns only
    # fraction control on the same shapes (a few rows, one column, one pixel)
    for (H, W) in [(1, 1), (1, 37), (41, 1), (2, 2), (3, 5), (3, 200)]:
        img = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        d = torch.from_numpy(img).cuda()
        for mode in (0, 1):
            for frac in (0.0, 0.3, 0.5, 1.0):
                got = sbs.boundaries(d, K=3, mode=mode, min_cc=1, frac=frac, seed=9).cpu().numpy().view(np.uint32)
                exp = oracle.boundaries(img, K=3, mode=mode, min_cc=1, frac=frac, seed=9)
                assert np.array_equal(got, exp), f"{H}x{W} mode {mode} frac {frac}"


def test_front_end_list_feeds_the_disparity_search(torch, sbs):
    """Frames from raw pixels to disparities on the device: front end, then SAD."""
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    L, R = torch.from_numpy(f.left).cuda(), torch.from_numpy(f.right).cuda()
    lst = sbs.boundaries(L, K=4, mode=0)
    d, c = sbs.sad_disparity(L, R, lst, spec.block, spec.dmax)
    idx = lst.cpu().numpy().view(np.uint32)
    ed, ec, _ = oracle.sad(f.left, f.right, idx, spec.block, spec.dmax)
    assert np.array_equal(d.cpu().numpy(), ed) and np.array_equal(c.cpu().numpy().view(np.uint32), ec)


def test_fraction_control_matches_oracle(torch, sbs):
    """Exactly round(f*W*H) pixels by the fixed ranking, for fractions that end
    inside the border columns, inside the kept pixels and among the other
    pixels (ranked by chessboard distance, then the seeded hash)."""
    cases = [("tsukuba_gray", 4, 0, 50), ("middlebury_rgb", 4, 0, 50), ("middlebury_rgb", 10, 1, 50)]
    for name, K, mode, min_cc in cases:
        spec = scenes.PRESETS[name]
        f = scenes.make_frame(spec)
        H, W = f.left.shape[:2]
        d = torch.from_numpy(np.ascontiguousarray(f.left)).cuda()
        _, kept_map = oracle.boundaries(f.left, K=K, mode=mode, min_cc=min_cc, frac=-1.0, return_map=True)
        kept_frac = kept_map[:, 1:-1].sum() / (W * H)
        fracs = [0.0, 0.5 / W, 2.0 / W + kept_frac / 2, 2.0 / W + kept_frac + 0.01, 0.18, 0.24, 0.7, 1.0]
        for frac in fracs:
            for seed in (spec.seed, 12345):
                got = sbs.boundaries(d, K=K, mode=mode, min_cc=min_cc, frac=frac, seed=seed).cpu().numpy().view(np.uint32)
                exp = oracle.boundaries(f.left, K=K, mode=mode, min_cc=min_cc, frac=frac, seed=seed)
                assert got.size == exp.size == min(W * H, int(np.floor(frac * (W * H) + 0.5))), f"{name} frac {frac}: sizes"
                assert np.array_equal(got, exp), f"{name} K{K} mode {mode} frac {frac} seed {seed}: lists differ"


def test_fraction_control_benchmark_frame(torch, sbs):
    """The 4096x2304 frame at 18%: the list the oracle's front end would give."""
    spec = scenes.PRESETS["uhd_rgb"]
    f = scenes.make_frame(spec)
    d = torch.from_numpy(np.ascontiguousarray(f.left)).cuda()
    got = sbs.boundaries(d, K=4, mode=0, min_cc=50, frac=0.18, seed=spec.seed).cpu().numpy().view(np.uint32)
    exp = oracle.boundaries(f.left, K=4, mode=0, min_cc=50, frac=0.18, seed=spec.seed)
    assert np.array_equal(got, exp)


def test_fraction_control_wide_rows_and_far_pixels(torch, sbs):
    """Fraction control into the distance class on rows wider than 4096 pixels
    (searched outwards from each pixel) and up to 4096 (range minima), on
    images whose few blobs leave most pixels far from any kept pixel."""
    rng = np.random.default_rng(11)
    for (H, W) in [(48, 4500), (96, 4096), (300, 257), (7, 4097)]:
        img = np.full((H, W, 3), 60, np.uint8)
        for _ in range(5):
            y, x = int(rng.integers(0, H)), int(rng.integers(0, W))
            img[max(0, y - 6):y + 6, max(0, x - 9):x + 9] = 200
        d = torch.from_numpy(img).cuda()
        for frac in (0.3, 0.6, 0.95):
            got = sbs.boundaries(d, K=2, mode=0, min_cc=1, frac=frac, seed=5).cpu().numpy().view(np.uint32)
            exp = oracle.boundaries(img, K=2, mode=0, min_cc=1, frac=frac, seed=5)
            assert np.array_equal(got, exp), f"{H}x{W} frac {frac}"


def test_kmeans_ties_on_few_grey_levels(torch, sbs):
    """Histograms of a few evenly spaced grey levels with equal or small
    counts: bins that lie exactly halfway between two centres (the tie goes
    to the centre tried first) and means that round alike in floating point,
    for K from 2 to 9, checked through the label image."""
    rng = np.random.default_rng(23)
    cases = []
    for step in range(1, 21):   # symmetric three- and five-level images: ties in the first pass
        for levels, K in ((3, 2), (5, 2), (5, 3), (5, 4)):
            base = int(rng.integers(0, 256 - step * (levels - 1)))
            cases.append((base + step * np.arange(levels), np.ones(levels, np.int64), K))
    for trial in range(60):
        levels = int(rng.integers(2, 7))
        step = int(rng.integers(1, 40))
        base = int(rng.integers(0, 256 - step * (levels - 1)))
        cases.append((base + step * np.arange(levels), rng.integers(1, 4, levels) * (1 if trial % 2 else 5),
                      int(rng.integers(2, 10))))
    for trial, (vals, counts, K) in enumerate(cases):
        pix = np.repeat(vals, counts).astype(np.uint8)
        side = int(np.ceil(np.sqrt(pix.size)))
        img = np.full(side * side, pix[-1], np.uint8)
        img[:pix.size] = pix
        img = img.reshape(side, side)
        d = torch.from_numpy(img).cuda()
        _, _, labels = sbs.boundaries(d, K=K, mode=1, min_cc=50, with_maps=True)
        exp = oracle_labels(img, K, 1)
        assert np.array_equal(labels.cpu().numpy(), exp), f"trial {trial}: levels {vals} counts {counts} K {K}"
