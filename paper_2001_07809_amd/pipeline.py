"""The whole method on the device, from a raw stereo pair to the selectively
blurred left image (arXiv 2001.07809, Sec. III), chaining the library's entry
points: lightness of both images, the front end on the left lightness, SAD
disparity at the listed pixels on the lightness images, reconstruction of the
dense map (Algorithms 1-2), then depth-based selective blurring (Eq. 1-2).

The paper's own setting (Table 3) is K = 10, 9x9 blocks, 'fill'/'remove'
refinement with the 4% component rule (mode 1), SAD on L* (one channel) and a
reconstruction threshold of 0 (Tsukuba) or 1. Every step runs in the
library's kernels; this module only passes device buffers along.
"""
from __future__ import annotations

from dataclasses import dataclass

import paper_2001_07809_amd as sbs


@dataclass
class PaperParams:
    K: int = 10
    mode: int = 1            # 1: fill/remove + 4% rule; 0: open/close + min_cc
    min_cc: int = 50
    block: int = 9
    dmax: int = 15
    threshold: int = 0       # reconstruction: disparity range above which the smaller value is taken
    ranges: tuple = ((0, 7),)   # in-focus disparity ranges (inclusive)
    sigma: float = 2.0


def depth_blur(left, right, p: PaperParams = PaperParams(), stream=None) -> dict:
    """left, right: device u8 images [H, W] or [H, W, 3]. Returns device
    tensors: 'l8' (left lightness), 'r8', 'list' (int32 raster indices),
    'disp' (u8 per list entry), 'cost' (int32), 'depth' (dense u8 [H, W]) and
    'blurred' (float32, the left image's shape)."""
    H, W = left.shape[0], left.shape[1]
    l8 = sbs.lightness(left, stream=stream)
    r8 = sbs.lightness(right, stream=stream)
    lst = sbs.boundaries(l8, K=p.K, mode=p.mode, min_cc=p.min_cc, stream=stream)
    disp, cost = sbs.sad_disparity(l8, r8, lst, p.block, p.dmax, stream=stream)
    depth = sbs.reconstruct(lst, disp, W, H, p.threshold, stream=stream)
    blurred = sbs.selective_blur(left, depth, p.ranges, p.sigma, stream=stream)
    return {"l8": l8, "r8": r8, "list": lst, "disp": disp, "cost": cost, "depth": depth, "blurred": blurred}


def bad_pixel_percent(computed, truth, mask=None, delta: float = 1.0) -> float:
    """Eq. 3: percentage of compared pixels whose |computed - truth| exceeds
    delta (1.0 in the paper). ``mask`` selects the compared pixels (host
    numpy arrays)."""
    import numpy as np
    c = np.asarray(computed, np.int32)
    t = np.asarray(truth, np.int32)
    bad = np.abs(c - t) > delta
    if mask is not None:
        bad = bad[np.asarray(mask, bool)]
    return 100.0 * float(bad.mean()) if bad.size else 0.0
