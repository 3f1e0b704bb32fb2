"""Pins for the oracle's SAD-WTA (Sec. III Disparity Measurement; Sec. II WTA).

The oracle is checked against things other than itself:
  * a hand-computed worked example (tests/golden/sad_hand_1row.json);
  * invariants the definition fixes (identical pair, global shift, constant
    images, channel replication, list order and subsets, dmax = 0);
  * a special case that reduces to a textbook routine (block 1 is pixel-wise
    absolute-difference WTA);
  * an independent algorithm (summed-area tables of the AD image);
  * an independent formulation by edge padding and slicing on tiny inputs;
  * the synthetic scenes' ground-truth disparities.
"""
import json
import os

import numpy as np
import pytest

import oracle
import scenes

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_computed_golden():
    g = json.load(open(os.path.join(GOLD, "sad_hand_1row.json")))
    L = np.array(g["left"], np.uint8).reshape(g["H"], g["W"])
    R = np.array(g["right"], np.uint8).reshape(g["H"], g["W"])
    for c in g["cases"]:
        d, cost, rc = oracle.sad(L, R, np.array([c["x"]], np.uint32), c["block"], c["dmax"])
        assert rc == 0
        assert (int(d[0]), int(cost[0])) == (c["disp"], c["cost"]), c["work"]


def _pad_ref(L, R, idx, block, dmax):
    """Edge padding + slicing formulation, written independently of the oracle's index clamping."""
    r = (block - 1) // 2
    if L.ndim == 2:
        L = L[:, :, None]
        R = R[:, :, None]
    H, W, C = L.shape
    P = r + dmax
    Lp = np.pad(L.astype(np.int64), ((r, r), (P, P), (0, 0)), mode="edge")
    Rp = np.pad(R.astype(np.int64), ((r, r), (P, P), (0, 0)), mode="edge")
    out_d, out_c = [], []
    for p in idx:
        y, x = divmod(int(p), W)
        lw = Lp[y:y + block, x + P - r:x + P + r + 1]
        costs = []
        for d in range(dmax + 1):
            rw = Rp[y:y + block, x + P - r - d:x + P + r + 1 - d]
            costs.append(int(np.abs(lw - rw).sum()))
        costs = np.array(costs)
        out_d.append(int(np.argmin(costs)))  # argmin returns the first minimum
        out_c.append(int(costs.min()))
    return np.array(out_d), np.array(out_c)


@pytest.mark.parametrize("C", [1, 3])
def test_tiny_sweep_against_padding_formulation(C):
    rng = np.random.default_rng(7 + C)
    for trial in range(60):
        W = int(rng.integers(1, 13))
        H = int(rng.integers(1, 13))
        block = int(rng.choice([1, 3, 5, 7]))
        dmax = int(rng.integers(0, W + 3))
        kind = trial % 4
        shape = (H, W) if C == 1 else (H, W, C)
        if kind == 0:
            L = rng.integers(0, 256, shape, dtype=np.uint8); R = rng.integers(0, 256, shape, dtype=np.uint8)
        elif kind == 1:
            L = np.full(shape, 77, np.uint8); R = np.full(shape, 80, np.uint8)
        elif kind == 2:
            L = (rng.integers(0, 2, shape) * 255).astype(np.uint8); R = (rng.integers(0, 2, shape) * 255).astype(np.uint8)
        else:  # few levels: many ties
            L = (rng.integers(0, 3, shape) * 10).astype(np.uint8); R = (rng.integers(0, 3, shape) * 10).astype(np.uint8)
        idx = np.arange(W * H, dtype=np.uint32)
        d, c, rc = oracle.sad(L, R, idx, block, dmax)
        rd, rcst = _pad_ref(L, R, idx, block, dmax)
        assert rc == 0
        np.testing.assert_array_equal(d, rd)
        np.testing.assert_array_equal(c, rcst)


def _texture(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 256, shape, dtype=np.uint8)


def test_identical_pair_gives_zero_everywhere():
    L = _texture((20, 33, 3), 1)
    idx = np.arange(20 * 33, dtype=np.uint32)
    d, c, _ = oracle.sad(L, L.copy(), idx, 7, 12)
    assert np.all(d == 0) and np.all(c == 0)


@pytest.mark.parametrize("s", [0, 1, 5, 11])
def test_global_shift_found_away_from_borders(s):
    block, dmax = 5, 12
    r = block // 2
    W, H = 48, 17
    big = _texture((H, W + s), 3)
    L = big[:, :W].copy()
    R = big[:, s:s + W].copy()          # R(x, y) = L(x + s, y)  ->  L(x) matches R(x - s)
    xs = np.arange(s + r, W - r)
    ys = np.arange(H)
    idx = (ys[:, None] * W + xs[None, :]).reshape(-1).astype(np.uint32)
    d, c, _ = oracle.sad(L, R, idx, block, dmax)
    assert np.all(d == s) and np.all(c == 0)


def test_constant_images_give_zero_disparity():
    L = np.full((9, 14), 200, np.uint8)
    R = np.full((9, 14), 13, np.uint8)
    idx = np.arange(9 * 14, dtype=np.uint32)
    d, c, _ = oracle.sad(L, R, idx, 3, 7)
    assert np.all(d == 0) and np.all(c == 9 * 187)


def test_channel_replication_triples_cost():
    g1 = _texture((15, 40), 4)
    g2 = _texture((15, 40), 5)
    idx = np.arange(15 * 40, dtype=np.uint32)
    d1, c1, _ = oracle.sad(g1, g2, idx, 5, 9)
    d3, c3, _ = oracle.sad(np.repeat(g1[:, :, None], 3, 2), np.repeat(g2[:, :, None], 3, 2), idx, 5, 9)
    np.testing.assert_array_equal(d1, d3)
    np.testing.assert_array_equal(c3, 3 * c1.astype(np.int64))


def test_list_order_subset_and_duplicates():
    L = _texture((25, 31, 3), 8)
    R = _texture((25, 31, 3), 9)
    idx = np.arange(25 * 31, dtype=np.uint32)
    d, c, _ = oracle.sad(L, R, idx, 5, 10)
    rng = np.random.default_rng(0)
    sub = rng.choice(idx, 300, replace=True).astype(np.uint32)   # shuffled, with repeats
    ds, cs, _ = oracle.sad(L, R, sub, 5, 10)
    np.testing.assert_array_equal(ds, d[sub])
    np.testing.assert_array_equal(cs, c[sub])


def test_dmax_zero_and_block_one_is_pixel_ad_wta():
    L = _texture((10, 20, 3), 10)
    R = _texture((10, 20, 3), 11)
    idx = np.arange(200, dtype=np.uint32)
    d, c, _ = oracle.sad(L, R, idx, 9, 0)
    assert np.all(d == 0)
    # block 1: cost(d) = sum_c |L(x, y, c) - R(max(x - d, 0), y, c)|, the pixel-wise AD cost.
    d1, c1, _ = oracle.sad(L, R, idx, 1, 6)
    Li = L.astype(np.int64)
    Ri = R.astype(np.int64)
    ad = np.stack([np.abs(Li - Ri[:, np.clip(np.arange(20) - dd, 0, 19)]).sum(-1) for dd in range(7)])
    exp_d = ad.argmin(0).reshape(-1)
    exp_c = ad.min(0).reshape(-1)
    np.testing.assert_array_equal(d1, exp_d)
    np.testing.assert_array_equal(c1, exp_c)


def test_out_of_range_index_is_flagged():
    L = _texture((4, 5), 12)
    d, c, rc = oracle.sad(L, L, np.array([0, 20, 19], np.uint32), 3, 2)
    assert rc == 5 and d[1] == 255 and c[1] == 0xFFFFFFFF and d[0] == 0 and d[2] == 0


def test_summed_area_table_agrees_on_tsukuba_shape():
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    lst = scenes.contour_list(f.rid, spec.frac, spec.seed)
    d, c, _ = oracle.sad(f.left, f.right, lst, spec.block, spec.dmax)
    d2, c2, _ = oracle.sad_sat(f.left, f.right, lst, spec.block, spec.dmax)
    np.testing.assert_array_equal(d, d2)
    np.testing.assert_array_equal(c, c2)


def test_summed_area_table_agrees_on_rgb_crop():
    spec = scenes.scaled(scenes.PRESETS["middlebury_rgb"], W=347, H=277)
    f = scenes.make_frame(spec)
    rng = np.random.default_rng(1)
    lst = np.sort(rng.choice(spec.W * spec.H, 3000, replace=False)).astype(np.uint32)
    d, c, _ = oracle.sad(f.left, f.right, lst, spec.block, spec.dmax)
    d2, c2, _ = oracle.sad_sat(f.left, f.right, lst, spec.block, spec.dmax)
    np.testing.assert_array_equal(d, d2)
    np.testing.assert_array_equal(c, c2)


def _qualifying(f, block):
    """Pixels whose whole window sits in one unoccluded region of constant disparity."""
    from scipy import ndimage as ndi
    r = block // 2
    gt = f.gt.astype(np.int32)
    rid = f.rid.astype(np.int32)
    same_gt = ndi.maximum_filter(gt, block, mode="constant", cval=10**6) == ndi.minimum_filter(gt, block, mode="constant", cval=-1)
    same_rid = ndi.maximum_filter(rid, block, mode="constant", cval=10**6) == ndi.minimum_filter(rid, block, mode="constant", cval=-10**6)
    vis = ndi.maximum_filter(f.occ, block, mode="constant", cval=1) == 0
    H, W = gt.shape
    ys, xs = np.mgrid[0:H, 0:W]
    inside = (xs - gt - r >= 0) & (xs + r <= W - 1) & (ys - r >= 0) & (ys + r <= H - 1)
    q = same_gt & same_rid & vis & inside
    return np.flatnonzero(q.reshape(-1)).astype(np.uint32)


def test_ground_truth_recovered_noise_free():
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    q = _qualifying(f, spec.block)
    assert q.size > 20000
    d, c, _ = oracle.sad(f.left, f.right, q, spec.block, spec.dmax)
    gt = f.gt.reshape(-1)[q]
    assert np.all(c == 0)
    assert np.all(d == gt)


def test_ground_truth_recovered_with_noise():
    spec = scenes.scaled(scenes.PRESETS["middlebury_rgb"], W=520, H=400, n_regions=10, dmax_regions=40)
    f = scenes.make_frame(spec)
    q = _qualifying(f, spec.block)
    rng = np.random.default_rng(2)
    q = np.sort(rng.choice(q, min(q.size, 6000), replace=False)).astype(np.uint32)
    d, c, _ = oracle.sad(f.left, f.right, q, spec.block, 63)
    gt = f.gt.reshape(-1)[q]
    assert np.mean(d == gt) >= 0.999
