"""The C-ABI library loads and exports every symbol include/sbs.h declares,
and rejects invalid arguments on the host before any device work (CPU only)."""
import ctypes
import os
import re

import pytest

import paper_2001_07809_amd as sbs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sbs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbs_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = sbs.lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert lib.sbs_abi_version() == 1


def _call(W=8, H=4, C=1, pitch=None, n=1, block=3, dmax=2, ptr=1):
    lib = sbs.lib()
    p = ctypes.c_void_p(ptr) if ptr else None
    return lib.sbs_sad_disparity(p, p, W, H, C, W * C if pitch is None else pitch, p, n, block, dmax,
                                 p, None, None, 0, None)


@pytest.mark.parametrize("kw,status", [
    (dict(W=0), 1), (dict(H=0), 1), (dict(C=2), 1), (dict(pitch=7), 1), (dict(block=4), 1),
    (dict(block=0), 1), (dict(dmax=-1), 1), (dict(dmax=256), 1), (dict(n=-1), 1), (dict(ptr=0), 1),
    (dict(block=129), 2),
])
def test_invalid_arguments_rejected_on_host(kw, status):
    assert _call(**kw) == status
    assert sbs.lib().sbs_last_error().decode() != ""


def test_empty_list_is_a_no_op_without_a_device():
    assert _call(n=0, ptr=0) == 0


def test_workspace_bytes_and_plans():
    f = sbs.Frame(1, 1, 100, 50, 3, 300, 1, 1000, 15, 31, 1, None)
    nb = sbs.workspace_bytes([f])
    assert nb > 100 * 50 * 4 * 3
    bad = sbs.Frame(1, 1, 100, 50, 2, 300, 1, 1000, 15, 31, 1, None)
    assert sbs.workspace_bytes([bad]) == 0
    assert sbs.workspace_bytes([f, f]) > nb
    with pytest.raises(sbs.SbsError):
        sbs.set_plan(chunk=12)
    with pytest.raises(sbs.SbsError):
        sbs.set_plan(cols_per_lane=8, chunk=16)   # 8 columns per lane only with 8-disparity chunks
    with pytest.raises(sbs.SbsError):
        sbs.set_plan(cols_per_lane=6)
    sbs.set_plan(cols_per_lane=8, chunk=8)
    assert sbs.get_plan(f)["cols_per_lane"] == 8
    sbs.set_plan(chunk=8, tile_rows=16)
    assert sbs.get_plan(f)["chunk"] == 8 and sbs.get_plan(f)["tile_rows"] == 16
    sbs.set_plan()
    assert sbs.get_plan(f)["chunk"] in (8, 16)


def test_injected_launch_failure_reported(monkeypatch):
    monkeypatch.setenv("SBS_TEST_FAIL", "launch")
    assert _call() == 4
    assert "injected" in sbs.lib().sbs_last_error().decode()
    monkeypatch.delenv("SBS_TEST_FAIL")
    assert _call(W=0) == 1


def _front(W=16, H=8, C=3, pitch=None, K=4, mode=0, min_cc=50, frac=-1.0, ptr=1, ws=None, wsptr=256):
    lib = sbs.lib()
    p = ctypes.c_void_p(ptr) if ptr else None
    w = ctypes.c_void_p(wsptr) if ptr else None
    need = lib.sbs_boundaries_workspace_bytes(W, H)
    return lib.sbs_boundaries(p, W, H, C, W * C if pitch is None else pitch, K, mode, min_cc, frac, 0, p, p, None,
                              None, w, need if ws is None else ws, None)


@pytest.mark.parametrize("kw", [dict(W=0), dict(H=0), dict(C=2), dict(pitch=10), dict(K=0), dict(K=65),
                                dict(mode=2), dict(min_cc=-1), dict(ptr=0), dict(ws=16), dict(frac=1.5),
                                dict(wsptr=256 + 16)])
def test_front_end_invalid_arguments_rejected_on_host(kw):
    assert _front(**kw) == 1
    assert sbs.lib().sbs_last_error().decode() != ""


def test_front_end_workspace_bytes():
    lib = sbs.lib()
    assert lib.sbs_boundaries_workspace_bytes(0, 5) == 0
    assert lib.sbs_boundaries_workspace_bytes(100, 50) >= 100 * 50 * 13
    assert lib.sbs_lightness(None, 4, 4, 3, 12, None, None) == 1


def test_noalloc_rejects_frames_beyond_the_scratch_on_host():
    # 8192x8192 RGB at block 31, dmax 127 needs more workspace than the fixed
    # scratch holds: refused before any device work.
    lib = sbs.lib()
    p = ctypes.c_void_p(1)
    st = lib.sbs_sad_disparity_noalloc(p, p, 8192, 8192, 3, 8192 * 3, p, 1 << 20, 31, 127, p, None, None)
    assert st == 3
    assert "scratch" in lib.sbs_last_error().decode()
    # invalid arguments still come first
    assert lib.sbs_sad_disparity_noalloc(p, p, 0, 8, 1, 8, p, 1, 3, 2, p, None, None) == 1
    assert lib.sbs_sad_disparity_noalloc(None, None, 8, 8, 1, 8, None, 0, 3, 2, None, None, None) == 0


def test_probe_rejects_bad_arguments_on_host():
    lib = sbs.lib()
    r, t = ctypes.c_double(), ctypes.c_double()
    assert lib.sbs_probe_sad_rate(0, 10, ctypes.byref(r), ctypes.byref(t)) == 1
    assert lib.sbs_probe_sad_rate(10, 0, ctypes.byref(r), ctypes.byref(t)) == 1
    assert lib.sbs_probe_sad_rate(10, 10, None, ctypes.byref(t)) == 1


def test_blur_rejects_bad_arguments_on_host():
    lib = sbs.lib()
    p = ctypes.c_void_p(256)
    rg = (ctypes.c_int32 * 2)(0, 10)
    need = lib.sbs_selective_blur_workspace_bytes(64, 32, 3)
    f = ctypes.c_float
    # geometry, ranges, sigma, workspace size and alignment: refused before any device work
    assert lib.sbs_selective_blur(p, 0, 32, 3, 192, p, rg, 1, f(2.0), p, p, need, None) == 1
    assert lib.sbs_selective_blur(p, 64, 32, 2, 192, p, rg, 1, f(2.0), p, p, need, None) == 1
    assert lib.sbs_selective_blur(p, 64, 32, 3, 100, p, rg, 1, f(2.0), p, p, need, None) == 1
    assert lib.sbs_selective_blur(p, 64, 32, 3, 192, p, rg, 17, f(2.0), p, p, need, None) == 1
    assert lib.sbs_selective_blur(p, 64, 32, 3, 192, p, rg, 1, f(0.0), p, p, need, None) == 1
    assert lib.sbs_selective_blur(p, 64, 32, 3, 192, p, rg, 1, f(2.0), p, p, need - 1, None) == 1
    assert lib.sbs_selective_blur(p, 64, 32, 3, 192, p, rg, 1, f(2.0), p, ctypes.c_void_p(258), need, None) == 1
    assert "aligned" in lib.sbs_last_error().decode()
    assert lib.sbs_selective_blur(p, 64, 32, 3, 192, p, rg, 1, f(30.0), p, p, need, None) == 2
