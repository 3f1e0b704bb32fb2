"""Serving loop: each request's result is identical alone and in the mix
(tolerance 0), admission respects the HBM budget, oversized requests are
refused, and the results match the oracle."""
import numpy as np
import pytest

import oracle
import scenes

pytestmark = pytest.mark.gpu

CLASSES = [
    scenes.SceneSpec(200, 150, 3, 5, 15, mean_shift=1, seed=7, block=11, dmax=15),
    scenes.SceneSpec(320, 240, 3, 8, 31, mean_shift=1, seed=8, block=15, dmax=31),
    scenes.SceneSpec(480, 272, 3, 10, 47, mean_shift=1, seed=9, block=21, dmax=47),
]


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2001_07809_amd as sbs
    from paper_2001_07809_amd.serve import BudgetError, Request, Server
    pool = []
    for ci, spec in enumerate(CLASSES):
        for s_i in range(2):
            sp = scenes.scaled(spec, seed=spec.seed * 10 + s_i)
            f = scenes.make_frame(sp)
            idx = scenes.contour_list(f.rid, 0.12 + 0.05 * s_i + 0.02 * ci, sp.seed)
            pool.append((sp, f, idx))
    return torch, sbs, Request, Server, BudgetError, pool


def _requests(env, n, arrivals):
    torch, sbs, Request, Server, BudgetError, pool = env
    reqs = []
    for i in range(n):
        sp, f, idx = pool[(i * 5) % len(pool)]
        reqs.append(Request(i, torch.from_numpy(f.left).cuda(), torch.from_numpy(f.right).cuda(),
                            torch.from_numpy(idx.view(np.int32)).cuda(), sp.block, sp.dmax, float(arrivals[i]),
                            f"{sp.W}x{sp.H}"))
    return reqs


def test_each_result_same_alone_and_in_the_mix(env):
    torch, sbs, Request, Server, BudgetError, pool = env
    reqs = _requests(env, 24, np.zeros(24))
    srv = Server(budget_bytes=64 << 20, max_inflight=2, max_batch=5)
    st = srv.run_trace(reqs)
    assert st["batches"] >= 5 and srv.peak_in_use <= srv.budget
    for r in reqs:
        d1, c1 = sbs.sad_disparity(r.left, r.right, r.idx, r.block, r.dmax)
        torch.cuda.synchronize()
        assert torch.equal(r.disp, d1) and torch.equal(r.cost, c1), f"request {r.rid}"
    # and against the oracle for one request of each class
    seen = set()
    for r in reqs:
        if r.klass in seen:
            continue
        seen.add(r.klass)
        d, c, _ = oracle.sad(r.left.cpu().numpy(), r.right.cpu().numpy(), r.idx.cpu().numpy().view(np.uint32),
                             r.block, r.dmax)
        np.testing.assert_array_equal(r.disp.cpu().numpy(), d)
        np.testing.assert_array_equal(r.cost.cpu().numpy().view(np.uint32), c)


def test_poisson_trace_and_budget(env):
    torch, sbs, Request, Server, BudgetError, pool = env
    rng = np.random.default_rng(3)
    arr = np.cumsum(rng.exponential(0.002, 30))
    reqs = _requests(env, 30, arr)
    budget = 6 << 20
    srv = Server(budget_bytes=budget, max_inflight=2, max_batch=64)
    st = srv.run_trace(reqs)
    assert st["requests"] == 30 and st["p99_ms"] >= st["p50_ms"] > 0
    assert srv.peak_in_use <= budget
    assert all(r.t_done >= r.t_admit >= r.arrival for r in reqs)
    tiny = Server(budget_bytes=1 << 16)
    with pytest.raises(BudgetError):
        tiny.submit(_requests(env, 1, [0.0])[0])


def test_raw_frames_through_the_device_front_end(env):
    """Requests that carry only their images: the server makes each list on the
    device (front end with fraction control) before the disparity search.
    Results equal the oracle's front end + SAD, alone and mixed with requests
    that bring their own lists."""
    torch, sbs, Request, Server, BudgetError, pool = env
    reqs = []
    for i in range(12):
        sp, f, idx = pool[i % len(pool)]
        L, R = torch.from_numpy(f.left).cuda(), torch.from_numpy(f.right).cuda()
        if i % 3 == 2:
            reqs.append(Request(i, L, R, torch.from_numpy(idx.view(np.int32)).cuda(), sp.block, sp.dmax, 0.0, "list"))
        else:
            reqs.append(Request(i, L, R, None, sp.block, sp.dmax, 0.0, "raw", frac=0.1 + 0.01 * i, seed=100 + i))
    srv = Server(budget_bytes=256 << 20, max_inflight=2, max_batch=4)
    srv.run_trace(reqs)
    for r in reqs:
        if r.klass != "raw":
            continue
        sp = pool[r.rid % len(pool)][0]
        Lh = r.left.cpu().numpy()
        exp_idx = oracle.boundaries(Lh, K=4, mode=0, min_cc=50, frac=r.frac, seed=r.seed)
        np.testing.assert_array_equal(r.idx.cpu().numpy().view(np.uint32), exp_idx)
        d, c, _ = oracle.sad(Lh, r.right.cpu().numpy(), exp_idx, r.block, r.dmax)
        np.testing.assert_array_equal(r.disp.cpu().numpy(), d)
        np.testing.assert_array_equal(r.cost.cpu().numpy().view(np.uint32), c)
        d1, c1 = sbs.sad_disparity(r.left, r.right, r.idx, r.block, r.dmax)
        torch.cuda.synchronize()
        assert torch.equal(r.disp, d1) and torch.equal(r.cost, c1)


def test_mixed_full_resolutions_alone_and_in_the_mix(env):
    """The serving mix's own request classes at their real sizes (640x480
    block 11 dmax 31, 1920x1080 block 21 dmax 63, 4096x2304 block 31 dmax
    127), each request with its own boundary fraction drawn from [0.12, 0.24]
    and its list from the device front end: every result equals the same
    request run alone, and sampled entries (first and last included) equal
    the oracle."""
    torch, sbs, Request, Server, BudgetError, pool = env
    rng = np.random.default_rng(105)
    reqs = []
    for ci, name in enumerate(("serve_vga", "serve_fhd", "serve_uhd")):
        spec = scenes.PRESETS[name]
        for k in range(3):
            sp = scenes.scaled(spec, seed=spec.seed + 1000 * ci + k)
            f = scenes.make_frame(sp)
            L, R = torch.from_numpy(f.left).cuda(), torch.from_numpy(f.right).cuda()
            frac = float(rng.uniform(0.12, 0.24))
            i = len(reqs)
            idx = sbs.boundaries(L, K=4, mode=0, min_cc=50, frac=frac, seed=sp.seed + i).clone()
            reqs.append(Request(i, L, R, idx, sp.block, sp.dmax, 0.0, name))
    order = rng.permutation(len(reqs))
    srv = Server(budget_bytes=2 << 30, max_inflight=2, max_batch=4)
    srv.run_trace([reqs[i] for i in order])
    for r in reqs:
        d1, c1 = sbs.sad_disparity(r.left, r.right, r.idx, r.block, r.dmax)
        torch.cuda.synchronize()
        assert torch.equal(r.disp, d1) and torch.equal(r.cost, c1), f"request {r.rid} ({r.klass})"
        idx = r.idx.cpu().numpy().view(np.uint32)
        pick = np.unique(np.concatenate([rng.choice(idx.size, 300, replace=False), [0, idx.size - 1]]))
        d, c, _ = oracle.sad(r.left.cpu().numpy(), r.right.cpu().numpy(), idx[pick], r.block, r.dmax)
        np.testing.assert_array_equal(r.disp.cpu().numpy()[pick], d, err_msg=f"request {r.rid} ({r.klass})")
        np.testing.assert_array_equal(r.cost.cpu().numpy().view(np.uint32)[pick], c)
