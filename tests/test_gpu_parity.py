"""GPU parity: the HIP path, called through the C-ABI, against the oracle.

Bar: bit-exact disparity AND cost (integer results). Small cases compare every
list entry with the oracle. At the full benchmark sizes the whole list is
checked against the GPU brute-force reference kernel (a separate code path),
and a random sample of entries against the oracle.
"""
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


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_gpu(torch, sbs, L, R, idx, block, dmax, path="tiled", **kw):
    Ld, Rd = dev(torch, L), dev(torch, R)
    Id = dev(torch, np.asarray(idx, np.uint32).view(np.int32))
    if path == "tiled":
        d, c = sbs.sad_disparity(Ld, Rd, Id, block, dmax, **kw)
    else:
        d, c = sbs.sad_disparity_ref(Ld, Rd, Id, block, dmax)
    torch.cuda.synchronize()
    return d.cpu().numpy(), c.cpu().numpy().view(np.uint32)


def assert_parity(got, exp, what=""):
    gd, gc = got
    ed, ec = exp[0], exp[1]
    bad = np.flatnonzero((gd != ed) | (gc != ec))
    assert bad.size == 0, f"{what}: {bad.size} mismatches, first at {bad[:5]}: gpu {gd[bad[:5]]}/{gc[bad[:5]]} oracle {ed[bad[:5]]}/{ec[bad[:5]]}"


def test_tiny_random_sweep(torch, sbs):
    rng = np.random.default_rng(11)
    for trial in range(40):
        W = int(rng.integers(1, 90))
        H = int(rng.integers(1, 70))
        C = int(rng.choice([1, 3]))
        block = int(rng.choice([1, 3, 5, 7, 9, 15, 31]))
        dmax = int(rng.integers(0, 80))
        shape = (H, W) if C == 1 else (H, W, C)
        L = rng.integers(0, 256, shape, dtype=np.uint8)
        R = rng.integers(0, 256, shape, dtype=np.uint8)
        if trial % 5 == 0:
            R = (R // 64 * 64).astype(np.uint8)     # coarse levels: many equal costs
            L = (L // 64 * 64).astype(np.uint8)
        idx = rng.permutation(W * H).astype(np.uint32)
        idx = np.concatenate([idx, idx[: max(1, idx.size // 7)]])   # shuffled, with duplicates
        exp = oracle.sad(L, R, idx, block, dmax)
        what = f"trial {trial} W{W} H{H} C{C} b{block} d{dmax}"
        assert_parity(run_gpu(torch, sbs, L, R, idx, block, dmax), exp, what + " tiled")
        assert_parity(run_gpu(torch, sbs, L, R, idx, block, dmax, path="ref"), exp, what + " ref")
        # ordered list, forced 8 columns per lane (and the unordered one under that plan)
        srt = np.unique(idx)
        try:
            sbs.set_plan(cols_per_lane=8, chunk=8, tile_rows=int(rng.choice([8, 32, 128])))
            assert_parity(run_gpu(torch, sbs, L, R, srt, block, dmax), oracle.sad(L, R, srt, block, dmax),
                          what + " ordered, 8 columns per lane")
            assert_parity(run_gpu(torch, sbs, L, R, idx, block, dmax), exp, what + " unordered, 8-column tiles")
        finally:
            sbs.set_plan()


def test_tsukuba_shape_full_list(torch, sbs):
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    idx = scenes.contour_list(f.rid, spec.frac, spec.seed)
    exp = oracle.sad(f.left, f.right, idx, spec.block, spec.dmax)
    assert_parity(run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax), exp, "tsukuba tiled")
    assert_parity(run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax, path="ref"), exp, "tsukuba ref")


def test_oracle_frontend_list(torch, sbs):
    # The list the oracle's own segmentation front end produces (K=4, open/close, CC >= 50, 18%).
    spec = scenes.PRESETS["tsukuba_gray"]
    f = scenes.make_frame(spec)
    idx = oracle.boundaries(f.left, K=4, mode=0, min_cc=50, frac=0.18, seed=spec.seed)
    exp = oracle.sad(f.left, f.right, idx, spec.block, spec.dmax)
    assert_parity(run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax), exp, "frontend list")
    vga = scenes.make_frame(scenes.PRESETS["serve_vga"])
    idx = oracle.boundaries(vga.left, K=4, mode=0, min_cc=50, frac=0.18, seed=5)
    exp = oracle.sad(vga.left, vga.right, idx, 11, 31)
    assert_parity(run_gpu(torch, sbs, vga.left, vga.right, idx, 11, 31), exp, "frontend list rgb")


def test_sorted_list_with_repeats(torch, sbs):
    # A list in non-decreasing order with every index twice, on a frame whose
    # tile rows hold every pixel (a tile row then has twice its width in list
    # entries): repeats must not take the ordered path, whose per-row ranges
    # count distinct entries.
    rng = np.random.default_rng(21)
    for C, W, H in ((3, 600, 40), (1, 1100, 24)):
        shape = (H, W) if C == 1 else (H, W, C)
        L = rng.integers(0, 256, shape, dtype=np.uint8)
        R = np.roll(L, -5, axis=1)
        base = np.arange(W * H, dtype=np.uint32)[rng.random(W * H) < 0.9]
        idx = np.sort(np.concatenate([base, base]))
        exp = oracle.sad(L, R, idx, 7, 40)
        try:
            for cpl, chunk in ((4, 8), (4, 16), (8, 8)):
                sbs.set_plan(cols_per_lane=cpl, chunk=chunk, tile_rows=32)
                assert_parity(run_gpu(torch, sbs, L, R, idx, 7, 40), exp,
                              f"sorted repeats C{C} {W}x{H} cpl{cpl} chunk{chunk}")
        finally:
            sbs.set_plan()


def test_middlebury_shape(torch, sbs):
    spec = scenes.PRESETS["middlebury_rgb"]
    f = scenes.make_frame(spec)
    idx = scenes.contour_list(f.rid, spec.frac, spec.seed)
    got = run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax)
    ref = run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax, path="ref")
    assert_parity(got, ref, "middlebury tiled vs ref (full list)")
    rng = np.random.default_rng(3)
    s = np.sort(rng.choice(idx.size, 20000, replace=False))
    exp = oracle.sad(f.left, f.right, idx[s], spec.block, spec.dmax)
    assert_parity((got[0][s], got[1][s]), exp, "middlebury sample vs oracle")


def test_uhd_shape_sampled(torch, sbs):
    spec = scenes.PRESETS["uhd_rgb"]
    f = scenes.make_frame(spec)
    idx = scenes.contour_list(f.rid, spec.frac, spec.seed)
    got = run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax)
    rng = np.random.default_rng(4)
    s = np.sort(rng.choice(idx.size, 1500, replace=False))
    exp = oracle.sad(f.left, f.right, idx[s], spec.block, spec.dmax)
    assert_parity((got[0][s], got[1][s]), exp, "uhd sample vs oracle")
    s2 = np.sort(rng.choice(idx.size, 60000, replace=False))
    ref = run_gpu(torch, sbs, f.left, f.right, idx[s2], spec.block, spec.dmax, path="ref")
    assert_parity((got[0][s2], got[1][s2]), ref, "uhd sample vs ref kernel")


def test_plans_agree(torch, sbs):
    spec = scenes.scaled(scenes.PRESETS["serve_fhd"], W=700, H=333)
    f = scenes.make_frame(spec)
    idx = scenes.contour_list(f.rid, 0.2, 1)
    base = None
    try:
        for cpl, chunk in ((4, 8), (4, 16), (8, 8)):
            for rows in (8, 16, 32, 64, 128, 256):
                sbs.set_plan(cols_per_lane=cpl, chunk=chunk, tile_rows=rows)
                got = run_gpu(torch, sbs, f.left, f.right, idx, spec.block, spec.dmax)
                if base is None:
                    base = got
                    exp = oracle.sad(f.left, f.right, idx, spec.block, spec.dmax)
                    assert_parity(got, exp, "plan base vs oracle")
                assert_parity(got, base, f"plan cols {cpl} chunk {chunk} rows {rows}")
    finally:
        sbs.set_plan()


def test_edge_cases(torch, sbs):
    rng = np.random.default_rng(5)
    # single pixel, single row, single column
    for (H, W) in [(1, 1), (1, 40), (37, 1)]:
        L = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        R = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
        idx = np.arange(W * H, dtype=np.uint32)
        exp = oracle.sad(L, R, idx, 5, 9)
        assert_parity(run_gpu(torch, sbs, L, R, idx, 5, 9), exp, f"{H}x{W}")
    L = rng.integers(0, 256, (50, 64), dtype=np.uint8)
    R = rng.integers(0, 256, (50, 64), dtype=np.uint8)
    idx = np.arange(50 * 64, dtype=np.uint32)
    for block, dmax in [(1, 0), (1, 40), (3, 0), (33, 255)]:
        exp = oracle.sad(L, R, idx, block, dmax)
        assert_parity(run_gpu(torch, sbs, L, R, idx, block, dmax), exp, f"b{block} d{dmax}")
    # largest block, largest dmax (sampled)
    L = rng.integers(0, 256, (200, 300, 3), dtype=np.uint8)
    R = rng.integers(0, 256, (200, 300, 3), dtype=np.uint8)
    idx = np.sort(rng.choice(200 * 300, 300, replace=False)).astype(np.uint32)
    exp = oracle.sad(L, R, idx, 127, 255)
    assert_parity(run_gpu(torch, sbs, L, R, idx, 127, 255), exp, "max block + dmax")
    # empty list
    d, c = run_gpu(torch, sbs, L, R, np.zeros(0, np.uint32), 15, 15)
    assert d.size == 0


def test_sparse_ordered_lists_with_long_gaps(torch, sbs):
    """Ordered lists whose entries sit many rows apart: the check writes the
    per-tile list ranges of the empty rows between two entries (and after the
    last one) with the whole wavefront, and every tile row still finds its
    entries. Also a list that is dense in one band and empty elsewhere, and
    lists at the image's first and last pixels."""
    rng = np.random.default_rng(12)
    H, W = 1300, 2100
    L = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    R = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    N = W * H
    band = np.arange(600 * W, 603 * W, 5)
    cases = {
        "seven spread": np.sort(rng.choice(N, 7, replace=False)),
        "first and last": np.array([0, N - 1]),
        "first only": np.array([0]),
        "last only": np.array([N - 1]),
        "one in the middle": np.array([N // 2 + 17]),
        "dense band": band,
        "band and corners": np.concatenate([[3], band, [N - 2]]),
    }
    for name, idx in cases.items():
        idx = idx.astype(np.uint32)
        exp = oracle.sad(L, R, idx, 9, 40)
        assert_parity(run_gpu(torch, sbs, L, R, idx, 9, 40), exp, name)


def test_row_pitch_and_no_cost_and_stream(torch, sbs):
    rng = np.random.default_rng(6)
    big = rng.integers(0, 256, (60, 120, 3), dtype=np.uint8)
    bigr = rng.integers(0, 256, (60, 120, 3), dtype=np.uint8)
    L = big[:, :97]
    R = bigr[:, :97]
    idx = np.arange(60 * 97, dtype=np.uint32)[::3].copy()
    exp = oracle.sad(np.ascontiguousarray(L), np.ascontiguousarray(R), idx, 7, 20)
    Ld = dev(torch, big)[:, :97]
    Rd = dev(torch, bigr)[:, :97]
    assert Ld.stride(0) == 360
    Id = dev(torch, idx.view(np.int32))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        d, c = sbs.sad_disparity(Ld, Rd, Id, 7, 20, stream=s)
        d2, c2 = sbs.sad_disparity(Ld, Rd, Id, 7, 20, stream=s, with_cost=False)
    s.synchronize()
    assert c2 is None
    assert_parity((d.cpu().numpy(), c.cpu().numpy().view(np.uint32)), exp, "pitched rows")
    np.testing.assert_array_equal(d2.cpu().numpy(), exp[0])


def test_out_of_range_index_reported(torch, sbs):
    rng = np.random.default_rng(7)
    L = rng.integers(0, 256, (20, 30), dtype=np.uint8)
    R = rng.integers(0, 256, (20, 30), dtype=np.uint8)
    idx = np.array([5, 600, 599, 10**6, 0], np.uint32)
    d, c = run_gpu(torch, sbs, L, R, idx, 5, 7)
    assert sbs.check_indices() == 5
    assert sbs.check_indices() == 0
    exp = oracle.sad(L, R, idx, 5, 7)
    assert_parity((d, c), exp, "out of range")
    assert d[1] == 255 and c[1] == 0xFFFFFFFF and d[3] == 255


def _video(spec, nframes):
    fr = scenes.video_fracs(spec, 0, nframes)
    left, right, lists = scenes.make_video(spec, 0, nframes, fr)
    return left, right, lists


def test_batched_equals_single_and_oracle(torch, sbs):
    spec = scenes.scaled(scenes.PRESETS["uhd_video"], W=640, H=360, n_regions=12)
    left, right, lists = _video(spec, 5)
    extra = scenes.make_frame(scenes.PRESETS["tsukuba_gray"])
    extra_idx = scenes.contour_list(extra.rid, 0.3, 9)
    frames = []
    keep = []
    for t in range(5):
        Ld, Rd, Id = dev(torch, left[t]), dev(torch, right[t]), dev(torch, lists[t].view(np.int32))
        keep += [Ld, Rd, Id]
        frames.append((Ld, Rd, Id, spec.block, spec.dmax))
    Ed, Erd, Eid = dev(torch, extra.left), dev(torch, extra.right), dev(torch, extra_idx.view(np.int32))
    frames.append((Ed, Erd, Eid, 15, 15))
    runner = sbs.BatchRunner(frames)
    runner.run()
    torch.cuda.synchronize()
    batched = [(runner.disp[i].cpu().numpy(), runner.cost[i].cpu().numpy().view(np.uint32)) for i in range(6)]
    for i in range(6):
        runner.disp[i].fill_(7)
    runner.run_per_frame()
    torch.cuda.synchronize()
    per = [(runner.disp[i].cpu().numpy(), runner.cost[i].cpu().numpy().view(np.uint32)) for i in range(6)]
    for t in range(5):
        exp = oracle.sad(left[t], right[t], lists[t], spec.block, spec.dmax)
        assert_parity(batched[t], exp, f"batched frame {t}")
        assert_parity(per[t], exp, f"per-frame frame {t}")
    exp = oracle.sad(extra.left, extra.right, extra_idx, 15, 15)
    assert_parity(batched[5], exp, "batched mixed frame")
    assert_parity(per[5], exp, "per-frame mixed frame")
    assert runner.check_indices() == 0


def test_graph_capture_replays(torch, sbs):
    spec = scenes.scaled(scenes.PRESETS["uhd_video"], W=512, H=288, n_regions=10)
    left, right, lists = _video(spec, 4)
    bufs = []
    frames = []
    for t in range(3):
        Ld, Rd, Id = dev(torch, left[t]), dev(torch, right[t]), dev(torch, lists[t].view(np.int32))
        bufs.append((Ld, Rd, Id))
        frames.append((Ld, Rd, Id, spec.block, spec.dmax))
    runner = sbs.BatchRunner(frames)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        runner.run(stream=s)          # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        runner.run()
    torch.cuda.synchronize()
    exp0 = oracle.sad(left[0], right[0], lists[0], spec.block, spec.dmax)
    exp3 = oracle.sad(left[3], right[3], lists[0], spec.block, spec.dmax)
    for rep in range(4):
        for i in range(3):
            runner.disp[i].fill_(0)
            runner.cost[i].fill_(-1)
        if rep == 2:
            # new pixels in frame 0's buffers (same list): the replay must recompute
            bufs[0][0].copy_(torch.from_numpy(left[3]))
            bufs[0][1].copy_(torch.from_numpy(right[3]))
        g.replay()
        torch.cuda.synchronize()
        got0 = (runner.disp[0].cpu().numpy(), runner.cost[0].cpu().numpy().view(np.uint32))
        assert_parity(got0, exp3 if rep >= 2 else exp0, f"replay {rep}")
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays


def test_saturated_sums_at_the_16_bit_accumulator_limit(torch, sbs):
    """Blocks on both sides of the packed-accumulator bound (2 * block * 255 * C
    <= 65535: two window columns added in 16-bit halves), images at 0 and 255
    so window column sums reach their maximum."""
    rng = np.random.default_rng(21)
    H, W = 180, 140
    for C, blocks in [(3, (41, 43, 83, 85, 87)), (1, (125, 127))]:
        shape = (H, W, C) if C == 3 else (H, W)
        L = (rng.integers(0, 2, shape) * 255).astype(np.uint8)
        L[:, : W // 2] = 255
        R = np.zeros(shape, np.uint8)
        R[H // 3:, :] = (rng.integers(0, 2, R[H // 3:].shape) * 255).astype(np.uint8)
        idx = np.sort(rng.choice(H * W, 400, replace=False)).astype(np.uint32)
        for block in blocks:
            exp = oracle.sad(L, R, idx, block, 20)
            assert exp[1].max() >= block * 255 * C // 2, "inputs must drive column sums near the limit"
            assert_parity(run_gpu(torch, sbs, L, R, idx, block, 20), exp, f"C{C} b{block} saturated")


def test_chunk16_all_instances(torch, sbs):
    """16-disparity chunks: ordered + packed frames run the 16-wide instance;
    unordered lists and 32-bit accumulators run two 8-wide passes per item.
    Partial last chunks (dmax + 1 not a multiple of 16, dmax < 8), 128-row
    tiles, single-frame and batched persistent launches."""
    rng = np.random.default_rng(12)
    cases = []
    for (H, W, C, block, dmax, order) in [(150, 260, 3, 15, 40, "sorted"), (150, 260, 3, 15, 40, "shuffled"),
                                          (140, 300, 3, 127, 20, "sorted"), (90, 200, 1, 9, 5, "sorted"),
                                          (90, 200, 1, 9, 127, "shuffled")]:
        shape = (H, W, C) if C == 3 else (H, W)
        L = rng.integers(0, 256, shape, dtype=np.uint8)
        R = np.roll(L, 3, axis=1)
        R[::7] = rng.integers(0, 256, R[::7].shape, dtype=np.uint8)
        idx = np.sort(rng.choice(H * W, H * W // 5, replace=False)).astype(np.uint32)
        if order == "shuffled":
            idx = np.concatenate([rng.permutation(idx), idx[:17]])
        cases.append((L, R, idx, block, dmax))
    try:
        for rows in (32, 128, 256):
            sbs.set_plan(chunk=16, tile_rows=rows)
            for (L, R, idx, block, dmax) in cases:
                exp = oracle.sad(L, R, idx, block, dmax)
                assert_parity(run_gpu(torch, sbs, L, R, idx, block, dmax), exp, f"chunk16 rows {rows} b{block} d{dmax}")
            frames = [(dev(torch, L), dev(torch, R), dev(torch, idx.view(np.int32)), block, dmax)
                      for (L, R, idx, block, dmax) in cases]
            runner = sbs.BatchRunner(frames)
            runner.run()
            torch.cuda.synchronize()
            for i, (L, R, idx, block, dmax) in enumerate(cases):
                exp = oracle.sad(L, R, idx, block, dmax)
                got = (runner.disp[i].cpu().numpy(), runner.cost[i].cpu().numpy().view(np.uint32))
                assert_parity(got, exp, f"chunk16 batched rows {rows} frame {i}")
    finally:
        sbs.set_plan()


def test_eight_columns_per_lane(torch, sbs):
    """Tiles of 512 window columns (8 per lane, 8-disparity chunks): ordered
    lists take the wide instance, with up to 128 listed pixels of a tile row
    in registers and the rest through the per-group path (dense rows); an
    unordered list runs the same tiles as narrower 4-column passes; frames
    whose window sums need 32 bits, and frames too wide for the packed row
    ranges (tile rows x W >= 2^23), fall back to 4 columns in the same call."""
    rng = np.random.default_rng(31)
    cases = []
    for (H, W, C, block, dmax, order) in [(150, 1100, 3, 31, 40, "sorted"), (150, 1100, 3, 31, 40, "shuffled"),
                                          (97, 523, 1, 9, 127, "sorted"), (70, 61, 3, 15, 8, "sorted"),
                                          (60, 900, 3, 45, 20, "sorted"), (33, 1300, 1, 3, 7, "dense"),
                                          (20, 2000, 3, 1, 0, "sorted")]:
        shape = (H, W, C) if C == 3 else (H, W)
        L = rng.integers(0, 256, shape, dtype=np.uint8)
        R = np.roll(L, 5, axis=1)
        R[::5] = rng.integers(0, 256, R[::5].shape, dtype=np.uint8)
        if order == "dense":   # whole rows listed: hundreds of entries per tile row
            rows = rng.choice(H, 6, replace=False)
            idx = np.sort(np.concatenate([np.arange(W) + y * W for y in rows])).astype(np.uint32)
        else:
            idx = np.sort(rng.choice(H * W, H * W // 5, replace=False)).astype(np.uint32)
        if order == "shuffled":
            idx = np.concatenate([rng.permutation(idx), idx[:23]])
        cases.append((L, R, idx, block, dmax))
    try:
        for rows in (8, 32, 128, 256):
            sbs.set_plan(cols_per_lane=8, chunk=8, tile_rows=rows)
            for (L, R, idx, block, dmax) in cases:
                exp = oracle.sad(L, R, idx, block, dmax)
                assert_parity(run_gpu(torch, sbs, L, R, idx, block, dmax), exp,
                              f"8 cols rows {rows} {L.shape} b{block} d{dmax}")
            frames = [(dev(torch, L), dev(torch, R), dev(torch, idx.view(np.int32)), block, dmax)
                      for (L, R, idx, block, dmax) in cases]
            runner = sbs.BatchRunner(frames)
            runner.run()
            torch.cuda.synchronize()
            for i, (L, R, idx, block, dmax) in enumerate(cases):
                exp = oracle.sad(L, R, idx, block, dmax)
                got = (runner.disp[i].cpu().numpy(), runner.cost[i].cpu().numpy().view(np.uint32))
                assert_parity(got, exp, f"8 cols batched rows {rows} frame {i}")
        # tile rows x W >= 2^23: the frame runs with 4 columns per lane
        H, W = 130, 66000
        L = rng.integers(0, 256, (H, W), dtype=np.uint8)
        R = np.roll(L, 2, axis=1)
        idx = np.sort(rng.choice(H * W, 3000, replace=False)).astype(np.uint32)
        sbs.set_plan(cols_per_lane=8, chunk=8, tile_rows=128)
        exp = oracle.sad(L, R, idx, 3, 9)
        assert_parity(run_gpu(torch, sbs, L, R, idx, 3, 9), exp, "wide frame fallback")
    finally:
        sbs.set_plan()


def test_long_list_on_a_wide_frame(torch, sbs):
    """A list of 2^24 + entries on a 70000-column frame: with 256-row tiles a
    row's list offset inside its tile would not fit the kernel's packed range
    (24 bits), so the frame runs with 128-row tiles; outputs checked on a
    sample against the oracle."""
    rng = np.random.default_rng(41)
    H, W = 300, 70000
    L = rng.integers(0, 256, (H, W), dtype=np.uint8)
    R = np.roll(L, 3, axis=1)
    keep = rng.random(H * W) < 0.82
    idx = np.flatnonzero(keep).astype(np.uint32)
    assert idx.size >= (1 << 24)
    try:
        for cpl in (4, 8):
            sbs.set_plan(cols_per_lane=cpl, chunk=8, tile_rows=256)
            d, c = run_gpu(torch, sbs, L, R, idx, 3, 7)
            pick = np.sort(rng.choice(idx.size, 3000, replace=False))
            pick = np.concatenate([pick, np.arange(200), idx.size - 1 - np.arange(200)])
            ed, ec, _ = oracle.sad(L, R, idx[pick], 3, 7)
            assert_parity((d[pick], c[pick]), (ed, ec), f"long list, {cpl} columns per lane")
    finally:
        sbs.set_plan()


def test_unaligned_caller_arrays(torch, sbs):
    """List and outputs at offsets that rule out the 16- and 4-byte vector
    paths of the list check and the finalize step (and at aligned offsets),
    lengths with a ragged tail of 1..3 entries, out-of-range indices inside
    and at the ends, ordered lists whose out-of-range indices form their
    tail (the finalize step stops at the first of them), unordered lists,
    with and without costs."""
    rng = np.random.default_rng(43)
    H, W = 70, 150
    L = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    R = np.roll(L, 4, axis=1)
    Ld, Rd = dev(torch, L), dev(torch, R)
    for order in ("sorted", "shuffled", "ordered tail"):
        for n in (1, 2, 3, 4, 5, 999, 1002, 1003):
            idx = np.sort(rng.choice(H * W, n, replace=False)).astype(np.uint32)
            if order == "ordered tail":   # still in raster order: indices >= W*H only at the end
                tail = np.array([H * W, H * W, H * W + 7, 0xFFFFFFF0], np.uint32)[: min(n, 1 + n % 4)]
                idx[n - tail.size:] = tail
            else:
                if order == "shuffled":
                    idx = rng.permutation(idx)
                idx[rng.integers(0, n)] = H * W + 7          # out of range
                if n > 2:
                    idx[0] = H * W
                    idx[-1] = 0xFFFFFFF0
            exp = oracle.sad(L, R, idx, 9, 20)
            for off_i, off_d, off_c in ((0, 0, 0), (1, 1, 1), (2, 3, 3), (3, 4, 2)):
                ib = dev(torch, np.concatenate([np.zeros(off_i, np.uint32), idx]).view(np.int32))[off_i:]
                out = torch.full((n + off_d,), 7, dtype=torch.uint8, device="cuda")[off_d:]
                cost = torch.full((n + off_c,), 7, dtype=torch.int32, device="cuda")[off_c:]
                d, c = sbs.sad_disparity(Ld, Rd, ib, 9, 20, out=out, cost=cost)
                torch.cuda.synchronize()
                what = f"{order} n {n} offsets {off_i},{off_d},{off_c}"
                assert_parity((d.cpu().numpy(), c.cpu().numpy().view(np.uint32)), exp, what)
                d2, c2 = sbs.sad_disparity(Ld, Rd, ib, 9, 20, out=out, with_cost=False)
                torch.cuda.synchronize()
                assert c2 is None and np.array_equal(d2.cpu().numpy(), exp[0]), what + " without costs"


def _image_at(torch, img, pitch, offset):
    """img (H, W, 3) on the device with rows `pitch` bytes apart, starting
    `offset` bytes into its allocation."""
    H, W, C = img.shape
    flat = np.zeros(offset + pitch * (H - 1) + W * C, np.uint8)
    for y in range(H):
        flat[offset + y * pitch: offset + y * pitch + W * C] = img[y].reshape(-1)
    return torch.from_numpy(flat).cuda().as_strided((H, W, C), (pitch, C, 1), offset)


def test_left_image_read_in_place(torch, sbs):
    """Tiles whose window lies inside the image read the caller's left RGB
    rows in place (4-byte-aligned base and pitch); the other tiles, and every
    tile of an image at an unaligned address or with a pitch that is not a
    multiple of 4, read the padded copy. The widths put a tile's window
    exactly at the last column that allows the in-place 16-byte loads (494
    for 4 columns per lane, 1006 for 8; block 9) and one column short of it;
    rows are pitched beyond W * 3 or packed; the first and last rows and
    columns are listed; ordered and unordered lists."""
    rng = np.random.default_rng(47)
    try:
        for (W, H, dmax, plan) in [(494, 23, 40, (4, 16)), (493, 23, 40, (4, 16)), (700, 19, 70, (4, 16)),
                                   (1006, 17, 20, (8, 8)), (1005, 17, 20, (8, 8))]:
            sbs.set_plan(cols_per_lane=plan[0], chunk=plan[1], tile_rows=8)
            L = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
            R = np.roll(L, 6, axis=1)
            R[::4] = rng.integers(0, 256, R[::4].shape, dtype=np.uint8)
            edge = np.concatenate([np.arange(2 * W), np.arange((H - 2) * W, H * W),
                                   np.arange(H) * W, np.arange(H) * W + W - 1])
            idx = np.unique(np.concatenate([rng.choice(H * W, H * W // 5, replace=False), edge])).astype(np.uint32)
            exp = oracle.sad(L, R, idx, 9, dmax)
            for order in ("sorted", "shuffled"):
                perm = np.arange(idx.size) if order == "sorted" else rng.permutation(idx.size)
                Id = dev(torch, idx[perm].view(np.int32))
                for (pitch, off) in ((3 * W, 0), (3 * W + 36, 0), (3 * W + 36, 1), (3 * W + 37, 0)):
                    Ld = _image_at(torch, L, pitch, off)
                    Rd = _image_at(torch, R, pitch, off)
                    d, c = sbs.sad_disparity(Ld, Rd, Id, 9, dmax)
                    torch.cuda.synchronize()
                    got = (d.cpu().numpy(), c.cpu().numpy().view(np.uint32))
                    assert_parity(got, (exp[0][perm], exp[1][perm]),
                                  f"W {W} plan {plan} {order} pitch {pitch} offset {off}")
    finally:
        sbs.set_plan()


def test_benchmark_configuration_sampled(torch, sbs):
    """Full-size frames of the benchmark's video (4096x2304 RGB, block 31,
    dmax 127) with the benchmark's lists: each frame's refined boundary set
    from the device front end (K = 4, open/close, components >= 50 px, border
    columns) cut to its per-frame fraction. Frame 0's list equals the
    oracle's front end. The batched persistent launch runs with the plan the
    benchmark's default comes to (16-disparity chunks, 128-row tiles, 16
    workgroups per CU), with the library's default for twelve frames, and
    with an autotuned plan: every frame is checked against the oracle on
    sampled entries (each frame's first and last entries included), and
    frame 0's whole list (about 1.7 M pixels, 2.2e8 evaluations) against the
    oracle in full."""
    spec = scenes.PRESETS["uhd_video"]
    F = 12
    fr = scenes.video_fracs(spec, 0, F)
    left, right, _ = scenes.make_video(spec, 0, F, with_lists=False)
    frames, keep, lists = [], [], []
    for t in range(F):
        Ld, Rd = dev(torch, left[t]), dev(torch, right[t])
        Id = sbs.boundaries(Ld, K=4, mode=0, min_cc=50, frac=float(fr[t]), seed=spec.seed + t).clone()
        keep += [Ld, Rd, Id]
        lists.append(Id.cpu().numpy().view(np.uint32))
        frames.append((Ld, Rd, Id, spec.block, spec.dmax))
    exp0_list = oracle.boundaries(left[0], K=4, mode=0, min_cc=50, frac=float(fr[0]), seed=spec.seed)
    assert np.array_equal(lists[0], exp0_list), "frame 0: device front-end list differs from the oracle's"
    rng = np.random.default_rng(17)
    try:
        for plan in ("benchmark", "default", "tuned"):
            sbs.set_plan()
            if plan == "benchmark":
                sbs.set_plan(cols_per_lane=4, chunk=16, tile_rows=128, waves_per_cu=16)
            runner = sbs.BatchRunner(frames)
            if plan == "tuned":
                runner.tune()
            runner.run()
            torch.cuda.synchronize()
            for t in range(F):
                n = lists[t].size
                pick = np.unique(np.concatenate([rng.choice(n, 250, replace=False), [0, n - 1]]))
                exp = oracle.sad(left[t], right[t], lists[t][pick], spec.block, spec.dmax)
                got = (runner.disp[t].cpu().numpy()[pick], runner.cost[t].cpu().numpy().view(np.uint32)[pick])
                assert_parity(got, exp, f"frame {t} ({plan} plan {runner.plan()})")
            if plan == "benchmark":
                exp = oracle.sad(left[0], right[0], lists[0], spec.block, spec.dmax)
                got = (runner.disp[0].cpu().numpy(), runner.cost[0].cpu().numpy().view(np.uint32))
                assert_parity(got, exp, f"frame 0, whole list of {lists[0].size} entries (benchmark plan)")
            assert runner.check_indices() == 0
            del runner
    finally:
        sbs.set_plan()
