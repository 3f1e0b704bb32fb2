"""GPU parity for the steps after the search: reconstruction (Algorithms 1-2,
bit-exact) and selective blur (Eq. 1-2, fp32 vs the oracle's fp64, |err| <= 1e-3)."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    import paper_2001_07809_amd as sbs
    return torch, sbs


@pytest.mark.parametrize("threshold", [0, 1, 4])
def test_reconstruct_matches_oracle(mods, threshold):
    torch, sbs = mods
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    idx = scenes.contour_list(f.rid, 0.18, 1)
    disp, _, _ = oracle.sad(f.left, f.right, idx, spec.block, spec.dmax)
    exp = oracle.reconstruct(idx, disp, spec.W, spec.H, threshold)
    got = sbs.reconstruct(torch.from_numpy(idx.view(np.int32)).cuda(), torch.from_numpy(disp).cuda(),
                          spec.W, spec.H, threshold)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), exp)


@pytest.mark.parametrize("W", [4096, 4097, 6000])
def test_reconstruct_row_fill_at_and_past_4096_columns(mods, W):
    """Rows of up to 4096 pixels keep a quarter row per wavefront in
    registers; wider rows walk it chunk by chunk. Runs of equal disparities
    between listed pixels, listed pixels at both row ends, empty rows."""
    torch, sbs = mods
    rng = np.random.default_rng(W)
    H = 24
    idx = np.sort(rng.choice(W * H, W * H // 9, replace=False))
    idx = np.unique(np.concatenate([idx, np.arange(H // 2) * W, np.arange(H // 2) * W + W - 1])).astype(np.uint32)
    idx = idx[(idx // W) % 7 != 3]                                # some rows without listed pixels
    disp = rng.integers(0, 4, idx.size).astype(np.uint8)           # few values: many equal neighbours
    for threshold in (0, 2):
        exp = oracle.reconstruct(idx, disp, W, H, threshold)
        got = sbs.reconstruct(torch.from_numpy(idx.view(np.int32)).cuda(), torch.from_numpy(disp).cuda(), W, H,
                              threshold)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), exp, err_msg=f"{W}x{H} t {threshold}")


def test_reconstruct_unordered_duplicates_and_edges(mods):
    torch, sbs = mods
    rng = np.random.default_rng(5)
    # the last two: a handful of listed pixels, so whole quarters of a row
    # (and whole rows) hold none and the nearest ones lie quarters apart
    for (W, H, n) in [(1, 1, 1), (1, 30, 6), (45, 1, 9), (300, 77, 4620), (4100, 3, 2460), (700, 9, 7),
                      (4100, 2, 3)]:
        idx = rng.integers(0, W * H + 3, n).astype(np.uint32)      # includes out-of-range entries
        disp = rng.integers(0, 6, n).astype(np.uint8)              # few values: many equal neighbours
        exp = oracle.reconstruct(idx, disp, W, H, 1)
        got = sbs.reconstruct(torch.from_numpy(idx.view(np.int32)).cuda(), torch.from_numpy(disp).cuda(), W, H, 1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), exp, err_msg=f"{W}x{H}")


def test_reconstruct_sparse_columns_across_segments(mods):
    """Few listed pixels on tall images: the column pass resolves rows from
    determined pixels many 16-row segments away (the segment scan carries the
    nearest value above and below across a thousand empty segments), in
    columns with one, several or no determined pixels; heights on and off a
    multiple of 16 and 64; and over a million rows, where segments grow past
    16 rows so that they fit the grid."""
    torch, sbs = mods
    rng = np.random.default_rng(6)
    for (W, H, n) in [(130, 700, 40), (3, 1000, 5), (64, 128, 10), (257, 64, 7), (90, 1, 3), (77, 641, 400),
                      (5, 20001, 6), (2, 9000, 1), (2, 1100003, 40000)]:
        idx = np.sort(rng.choice(W * H, n, replace=False)).astype(np.uint32)
        disp = rng.integers(0, 40, n).astype(np.uint8)
        for threshold in (0, 3):
            exp = oracle.reconstruct(idx, disp, W, H, threshold)
            got = sbs.reconstruct(torch.from_numpy(idx.view(np.int32)).cuda(), torch.from_numpy(disp).cuda(), W, H,
                                  threshold)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(got.cpu().numpy(), exp, err_msg=f"{W}x{H} n {n} t {threshold}")


@pytest.mark.parametrize("C,sigma", [(1, 0.8), (3, 1.5), (3, 4.0), (3, 4.6), (1, 5.0), (3, 5.0)])
def test_blur_matches_oracle(mods, C, sigma):
    torch, sbs = mods
    rng = np.random.default_rng(7)
    shape = (70, 93) if C == 1 else (70, 93, 3)
    img = rng.integers(0, 256, shape, dtype=np.uint8)
    depth = rng.integers(0, 40, (70, 93), dtype=np.uint8)
    ranges = [(3, 9), (30, 35)]
    exp = oracle.blur(img, depth, ranges, sigma)
    got = sbs.selective_blur(torch.from_numpy(img).cuda(), torch.from_numpy(depth).cuda(), ranges, sigma)
    torch.cuda.synchronize()
    np.testing.assert_allclose(got.cpu().numpy(), exp, atol=1e-3, rtol=0)

@pytest.mark.parametrize("W", [300, 298])
@pytest.mark.parametrize("sigma", [2.0, 4.6])
def test_blur_pitched_rows_over_many_tiles(mods, sigma, W):
    """An RGB image inside wider rows (pitch > W * 3), several 64 x 32 tiles
    with partial ones at the right and bottom, the largest radius the tiled
    kernel takes (14 at sigma 4.6) and a common one (6 at sigma 2); a width
    that is not a multiple of 4 (depth rows not word-aligned) with aligned
    image rows."""
    torch, sbs = mods
    rng = np.random.default_rng(11)
    H = 150
    wide = rng.integers(0, 256, (H, 320, 3), dtype=np.uint8)
    img = np.ascontiguousarray(wide[:, :W])
    depth = rng.integers(0, 60, (H, W), dtype=np.uint8)
    ranges = [(0, 20)]
    exp = oracle.blur(img, depth, ranges, sigma)
    dev = torch.from_numpy(wide).cuda()[:, :W]
    assert dev.stride(0) == 960
    got = sbs.selective_blur(dev, torch.from_numpy(depth).cuda(), ranges, sigma)
    torch.cuda.synchronize()
    np.testing.assert_allclose(got.cpu().numpy(), exp, atol=1e-3, rtol=0)



@pytest.mark.parametrize("C,sigma", [(3, 0.3), (1, 2.3), (3, 2.3), (3, 2.6), (1, 2.6)])
@pytest.mark.parametrize("H,W", [(1, 70), (37, 131), (96, 256), (33, 65), (70, 301)])
def test_blur_matrix_core_radii(mods, C, sigma, H, W):
    """Radii 1, 7 and 8 (the largest the matrix-core path takes): one-row
    images, partial tiles, odd widths (rows not 4-byte aligned: word loads
    from the boundary below, shifted into place, for interior tiles at 301
    columns; clamped bytes for the edge tiles) and aligned widths."""
    torch, sbs = mods
    rng = np.random.default_rng(17)
    shape = (H, W) if C == 1 else (H, W, C)
    img = rng.integers(0, 256, shape, dtype=np.uint8)
    depth = rng.integers(0, 40, (H, W), dtype=np.uint8)
    ranges = [(3, 9), (30, 35)]
    exp = oracle.blur(img, depth, ranges, sigma)
    got = sbs.selective_blur(torch.from_numpy(img).cuda(), torch.from_numpy(depth).cuda(), ranges, sigma)
    torch.cuda.synchronize()
    np.testing.assert_allclose(got.cpu().numpy(), exp, atol=1e-3, rtol=0)


def test_blur_full_frame_4096x2304(mods):
    """Every output of a 4096x2304 RGB frame at sigma 2 (radius 6, the paper
    chain's setting) against the oracle: random bytes (the worst case for the
    fp16 splits: every tap sees a full-range value), a depth map of 64 x 32
    blocks in focus, out of focus and mixed."""
    torch, sbs = mods
    rng = np.random.default_rng(19)
    H, W = 2304, 4096
    img = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    kinds = rng.integers(0, 3, (H // 32, W // 64))
    depth = rng.integers(0, 128, (H, W), dtype=np.uint8)
    full = np.repeat(np.repeat(kinds, 32, axis=0), 64, axis=1)
    depth[full == 0] = 10
    depth[full == 1] = 100
    ranges = [(0, 42)]
    exp = oracle.blur(img, depth, ranges, 2.0)
    got = sbs.selective_blur(torch.from_numpy(img).cuda(), torch.from_numpy(depth).cuda(), ranges, 2.0)
    torch.cuda.synchronize()
    err = np.abs(got.cpu().numpy().astype(np.float64) - exp)
    assert err.max() <= 1e-3, f"max |err| {err.max():.3g}"
    # in-focus pixels are copied exactly
    keep = (depth <= 42)
    assert np.array_equal(got.cpu().numpy()[keep], img[keep].astype(np.float32))


@pytest.mark.parametrize("C,sigma", [(3, 2.0), (1, 1.2), (3, 4.6)])
def test_blur_tiles_in_focus_and_aligned_rows(mods, C, sigma):
    """Depth maps made of 64 x 32 blocks (the blur's tiles): whole tiles in
    focus (their pixels converted only), whole tiles out of focus, and mixed
    tiles; images with 4-byte-aligned rows wide enough for interior tiles
    (read as aligned dwords) as well as the clamped edge tiles."""
    torch, sbs = mods
    rng = np.random.default_rng(13)
    H, W = 200, 512
    shape = (H, W) if C == 1 else (H, W, C)
    img = rng.integers(0, 256, shape, dtype=np.uint8)
    blocks = rng.integers(0, 3, ((H + 31) // 32, W // 64))
    depth = np.empty((H, W), np.uint8)
    for by in range(blocks.shape[0]):
        for bx in range(blocks.shape[1]):
            sl = (slice(32 * by, 32 * by + 32), slice(64 * bx, 64 * bx + 64))
            kind = blocks[by, bx]
            if kind == 0:      # in focus
                depth[sl] = 5
            elif kind == 1:    # blurred
                depth[sl] = 50
            else:              # mixed
                depth[sl] = rng.choice([5, 50], depth[sl].shape)
    ranges = [(0, 10)]
    exp = oracle.blur(img, depth, ranges, sigma)
    got = sbs.selective_blur(torch.from_numpy(img).cuda(), torch.from_numpy(depth).cuda(), ranges, sigma)
    torch.cuda.synchronize()
    np.testing.assert_allclose(got.cpu().numpy(), exp, atol=1e-3, rtol=0)


@pytest.mark.parametrize("sigma", [2.0, 4.6])
def test_blur_no_ranges_and_all_in_focus(mods, sigma):
    """No range of interest (every pixel blurred), several ranges at once,
    and one range that covers every depth (every tile copied through), on
    the matrix-core path (sigma 2) and the fp32 tile path (sigma 4.6)."""
    torch, sbs = mods
    rng = np.random.default_rng(29)
    H, W = 100, 333
    img = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    depth = rng.integers(0, 64, (H, W), dtype=np.uint8)
    for ranges in ([], [(0, 3), (10, 12), (20, 20), (40, 63)], [(0, 255)]):
        exp = oracle.blur(img, depth, ranges, sigma)
        got = sbs.selective_blur(torch.from_numpy(img).cuda(), torch.from_numpy(depth).cuda(), ranges, sigma)
        torch.cuda.synchronize()
        np.testing.assert_allclose(got.cpu().numpy(), exp, atol=1e-3, rtol=0, err_msg=f"ranges {ranges}")
        if ranges == [(0, 255)]:
            assert np.array_equal(got.cpu().numpy(), img.astype(np.float32))
