"""Autotuner: sbs_tune picks a plan, writes it to a JSON cache, the cache
loads back, later calls use it, and results do not depend on the plan."""
import json

import numpy as np
import pytest

import scenes

pytestmark = pytest.mark.gpu


def test_tune_cache_roundtrip(tmp_path):
    import torch
    import paper_2001_07809_amd as sbs
    spec = scenes.scaled(scenes.PRESETS["uhd_video"], W=700, H=400, n_regions=10)
    fr = scenes.video_fracs(spec, 0, 3)
    left, right, lists = scenes.make_video(spec, 0, 3, fr)
    frames = [(torch.from_numpy(left[t]).cuda(), torch.from_numpy(right[t]).cuda(),
               torch.from_numpy(lists[t].view(np.int32)).cuda(), spec.block, spec.dmax) for t in range(3)]
    runner = sbs.BatchRunner(frames)
    runner.run()
    torch.cuda.synchronize()
    before = [d.clone() for d in runner.disp]
    cache = tmp_path / "tuning.json"
    sbs.tune(list(runner.desc), str(cache))
    data = json.loads(cache.read_text())
    # the cache holds every plan tuned in this process; this batch's key ends
    # with its frame count rounded up to a power of two
    mine = {k: v for k, v in data.items() if k.startswith("gfx950/700x400x3/b31/d127/")}
    assert len(mine) == 1
    (key, plan), = mine.items()
    assert key.endswith("/nf4") and plan["chunk"] in (8, 16)
    sbs.load_tuning(str(cache))
    assert runner.plan() == plan
    for d in runner.disp:
        d.fill_(0)
    runner.run()
    torch.cuda.synchronize()
    for a, b in zip(before, runner.disp):
        assert torch.equal(a, b)


def test_tune_single_frame(tmp_path):
    """One frame is tuned on the single-frame launch sequence: its key ends
    with /nf1, the persistent grid size keeps its default, sad_disparity
    picks the stored plan up, and its output does not change."""
    import torch
    import paper_2001_07809_amd as sbs
    spec = scenes.scaled(scenes.PRESETS["uhd_video"], W=640, H=360, n_regions=8)
    fr = scenes.video_fracs(spec, 0, 1)
    left, right, lists = scenes.make_video(spec, 0, 1, fr)
    L = torch.from_numpy(left[0]).cuda()
    R = torch.from_numpy(right[0]).cuda()
    idx = torch.from_numpy(lists[0].view(np.int32)).cuda()
    d0, c0 = sbs.sad_disparity(L, R, idx, spec.block, spec.dmax)
    torch.cuda.synchronize()
    d0, c0 = d0.clone(), c0.clone()
    out = torch.empty_like(d0)
    frame = sbs.make_frame(L, R, idx, spec.block, spec.dmax, out, None)
    cache = tmp_path / "tuning.json"
    sbs.tune([frame], str(cache))
    data = json.loads(cache.read_text())
    mine = {k: v for k, v in data.items() if k.startswith("gfx950/640x360x3/")}
    assert len(mine) == 1
    (key, plan), = mine.items()
    assert key.endswith("/nf1") and plan["waves_per_cu"] == 16
    assert sbs.get_plan(frame) == plan
    d1, c1 = sbs.sad_disparity(L, R, idx, spec.block, spec.dmax)
    torch.cuda.synchronize()
    assert torch.equal(d0, d1) and torch.equal(c0, c1)
    assert torch.equal(out, d0)
