"""The fixed-scratch entry point (sbs_sad_disparity_noalloc) through the C-ABI
against sbs_sad_disparity on the same inputs: bit-exact disparity and cost, on
calls in a row that leave the scratch holding the previous call's contents
(each later call smaller than the one before it)."""
import numpy as np
import pytest

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


def _case(torch, spec, frac, shuffle_seed=None):
    f = scenes.make_frame(spec)
    idx = scenes.contour_list(f.rid, frac, spec.seed)
    if shuffle_seed is not None:   # unordered list with repeats: the pixel-map path
        rng = np.random.default_rng(shuffle_seed)
        idx = rng.permutation(np.concatenate([idx, idx[: idx.size // 5]])).astype(np.uint32)
    L = torch.from_numpy(f.left).cuda()
    R = torch.from_numpy(f.right).cuda()
    I = torch.from_numpy(idx.view(np.int32)).cuda()
    return L, R, I, spec


def _both(torch, sbs, L, R, I, spec):
    d0, c0 = sbs.sad_disparity(L, R, I, spec.block, spec.dmax)
    d1, c1 = sbs.sad_disparity_noalloc(L, R, I, spec.block, spec.dmax)
    torch.cuda.synchronize()
    return (d0.cpu().numpy(), c0.cpu().numpy()), (d1.cpu().numpy(), c1.cpu().numpy())


def test_noalloc_equals_workspace_entry_point_on_calls_in_a_row(torch, sbs):
    cases = [
        ("4096x2304 RGB, unordered list with repeats", scenes.PRESETS["uhd_rgb"], 0.24, 5),
        ("1390x1110 RGB, ordered list", scenes.PRESETS["middlebury_rgb"], 0.18, None),
        ("384x288 gray, unordered list", scenes.PRESETS["tsukuba_gray"], 0.18, 9),
        ("384x288 gray, ordered list", scenes.PRESETS["tsukuba_gray"], 0.12, None),
    ]
    for what, spec, frac, shuffle in cases:
        print(f"noalloc case: {what}", flush=True)
        L, R, I, spec = _case(torch, spec, frac, shuffle)
        (d0, c0), (d1, c1) = _both(torch, sbs, L, R, I, spec)
        bad = np.flatnonzero((d0 != d1) | (c0 != c1))
        assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}"
