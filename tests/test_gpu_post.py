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


def test_reconstruct_unordered_duplicates_and_edges(mods):
    torch, sbs = mods
    rng = np.random.default_rng(5)
    for (W, H) in [(1, 1), (1, 30), (45, 1), (300, 77), (4100, 3)]:
        n = max(1, W * H // 5)
        idx = rng.integers(0, W * H + 3, n).astype(np.uint32)      # includes out-of-range entries
        disp = rng.integers(0, 6, n).astype(np.uint8)              # few values: many equal neighbours
        exp = oracle.reconstruct(idx, disp, W, H, 1)
        got = sbs.reconstruct(torch.from_numpy(idx.view(np.int32)).cuda(), torch.from_numpy(disp).cuda(), W, H, 1)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), exp, err_msg=f"{W}x{H}")


@pytest.mark.parametrize("C,sigma", [(1, 0.8), (3, 1.5), (3, 4.0)])
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
