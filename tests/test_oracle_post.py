"""Pins for the oracle's disparity-map reconstruction (Sec. III, Algorithm 1
'fill' along scan lines, Algorithm 2 'peek' along columns) and depth-based
selective blurring (Sec. III, Eq. 1-2)."""
import numpy as np
from scipy import ndimage as ndi

import oracle


def _sparse(points, W):
    idx = np.array([y * W + x for (y, x, d) in points], np.uint32)
    disp = np.array([d for (y, x, d) in points], np.uint8)
    return idx, disp


def test_fill_between_equal_boundary_disparities():
    # Row 0: boundary at x=1 (d=5) and x=6 (d=5) -> x=2..5 filled with 5 by Algorithm 1.
    # Row 1: boundary at x=1 (d=5) and x=6 (d=7) -> nothing filled in that row.
    W, H = 8, 2
    idx, disp = _sparse([(0, 1, 5), (0, 6, 5), (1, 1, 5), (1, 6, 7)], W)
    out = oracle.reconstruct(idx, disp, W, H, threshold=0)
    assert list(out[0, 1:7]) == [5, 5, 5, 5, 5, 5]
    # Row 1 x=2..5 are undetermined after stage 1; the peek looks along columns:
    # above (row 0) holds 5, nothing below -> one-sided -> 5.
    assert list(out[1, 2:6]) == [5, 5, 5, 5]


def test_peek_threshold_smaller_or_mean():
    # Column 0: known 4 at row 0, known 9 at row 4; rows 1..3 undetermined.
    W, H = 1, 5
    idx, disp = _sparse([(0, 0, 4), (4, 0, 9)], W)
    # range 5 > threshold 1 -> the smaller value
    out = oracle.reconstruct(idx, disp, W, H, threshold=1)
    assert list(out[:, 0]) == [4, 4, 4, 4, 9]
    # range 5 <= threshold 5 -> mean rounded half up: (4 + 9 + 1) // 2 = 7
    out = oracle.reconstruct(idx, disp, W, H, threshold=5)
    assert list(out[:, 0]) == [4, 7, 7, 7, 9]


def test_peek_reads_only_fill_output_and_empty_columns():
    W, H = 3, 4
    idx, disp = _sparse([(0, 0, 2), (0, 2, 2), (3, 0, 6)], W)
    out = oracle.reconstruct(idx, disp, W, H, threshold=0)
    # row 0 filled by Alg. 1: (0,1) = 2; column 1 then has only row 0 known -> 2 below it
    assert out[0, 1] == 2 and list(out[1:, 1]) == [2, 2, 2]
    # column 0: 2 above, 6 below, range 4 > 0 -> smaller = 2
    assert list(out[1:3, 0]) == [2, 2]
    # column 2: only row 0 known -> 2
    assert list(out[:, 2]) == [2, 2, 2, 2]
    empty = oracle.reconstruct(np.zeros(0, np.uint32), np.zeros(0, np.uint8), 4, 3, 0)
    assert np.all(empty == 0)


def test_blur_matches_separable_gaussian_and_keeps_in_focus_pixels():
    rng = np.random.default_rng(0)
    img = rng.integers(0, 256, (40, 50, 3), dtype=np.uint8)
    depth = rng.integers(0, 30, (40, 50), dtype=np.uint8)
    ranges = [(5, 9), (20, 22)]
    sigma = 1.5
    out = oracle.blur(img, depth, ranges, sigma)
    keep = ((depth >= 5) & (depth <= 9)) | ((depth >= 20) & (depth <= 22))
    np.testing.assert_array_equal(out[keep], img[keep].astype(np.float32))
    # Eq. 1-2 on a (2*ceil(3 sigma)+1)^2 support equals scipy's separable filter
    # with the same radius (truncate = ceil(3 sigma) / sigma), replicate border.
    rad = int(np.ceil(3 * sigma))
    ref = np.stack([ndi.gaussian_filter(img[..., c].astype(np.float64), sigma, mode="nearest",
                                        truncate=rad / sigma) for c in range(3)], -1)
    np.testing.assert_allclose(out[~keep], ref[~keep], atol=1e-3)
    const = np.full((10, 12), 77, np.uint8)
    cb = oracle.blur(const, np.zeros((10, 12), np.uint8), [(1, 3)], 2.0)
    np.testing.assert_allclose(cb, 77.0, atol=1e-4)
