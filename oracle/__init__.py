"""Oracle: plain CPU implementation of the boundary-pixel SAD disparity path.

THIS IS TEST INFRASTRUCTURE. Only the tests, ``__graft_entry__.smoke()`` and
the benchmark's ``cpu_baseline`` leg may import it. The HIP product path never
imports it, and the two share no code.

The C++ source is ``oracle.cpp``. Each function there cites the passage of
the paper (arXiv 2001.07809) that it follows. ``build()`` compiles it to
``liboracle.so`` in this folder.

Parity status: every function is pinned by the CPU tests
(``tests/test_oracle_*.py``), the K-means start by hand-worked histograms and
the fraction-control ranking (``fraction_select``) by library routines. The lightness rounding in ``lightness()`` is
pinned only at known values and by monotonicity, because the paper's colour
transform reference is lost. It affects which pixels a list holds, never a
SAD value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC"]


def build() -> str:
    """Compile liboracle.so (always recompiles)."""
    cmd = ["g++", *CFLAGS, os.path.join(_HERE, "oracle.cpp"), "-o", _SO + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    V, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "oracle_lightness": ([V, I32, I32, I32, I64, V], None),
        "oracle_histogram": ([V, I64, V], None),
        "oracle_kmeans_bins": ([V, I32, V, V, V], ctypes.c_int),
        "oracle_label_pixels": ([V, I64, V, V], None),
        "oracle_label_open_close": ([V, I32, I32, V], None),
        "oracle_erode3": ([V, I32, I32, V], None),
        "oracle_dilate3": ([V, I32, I32, V], None),
        "oracle_boundary": ([V, I32, I32, V], None),
        "oracle_fill": ([V, I32, I32, V], None),
        "oracle_remove": ([V, I32, I32, V], None),
        "oracle_components": ([V, I32, I32, V, V], I64),
        "oracle_cc_filter": ([V, I32, I32, I32, I64, D, V], None),
        "oracle_boundaries": ([V, I32, I32, I32, I64, I32, I32, I64, D, U64, V, I64, V], I64),
        "oracle_fraction_select": ([V, I32, I32, D, U64, V, I64], I64),
        "oracle_sad": ([V, V, I32, I32, I32, I64, V, I64, I32, I32, V, V, I32], ctypes.c_int),
        "oracle_sad_sat": ([V, V, I32, I32, I32, I64, V, I64, I32, I32, V, V], ctypes.c_int),
        "oracle_reconstruct": ([V, V, I64, I32, I32, I32, V], None),
        "oracle_blur": ([V, I32, I32, I32, I64, V, V, I32, D, V], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _img(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    H, W = a.shape[:2]
    C = 1 if a.ndim == 2 else a.shape[2]
    return a, W, H, C, W * C


def lightness(img: np.ndarray) -> np.ndarray:
    img, W, H, C, pitch = _img(img)
    out = np.empty((H, W), np.uint8)
    _load().oracle_lightness(_p(img), W, H, C, pitch, _p(out))
    return out


def histogram(L8: np.ndarray) -> np.ndarray:
    L8 = np.ascontiguousarray(L8, dtype=np.uint8)
    h = np.empty(256, np.int64)
    _load().oracle_histogram(_p(L8), L8.size, _p(h))
    return h


def kmeans_bins(hist: np.ndarray, K: int):
    """Returns (bin_label[256] int32, centres as float, passes)."""
    hist = np.ascontiguousarray(hist, dtype=np.int64)
    bl = np.empty(256, np.int32)
    cS = np.zeros(K, np.int64)
    cN = np.ones(K, np.int64)
    passes = _load().oracle_kmeans_bins(_p(hist), K, _p(bl), _p(cS), _p(cN))
    return bl, cS, cN, passes


def label_pixels(L8: np.ndarray, bin_label: np.ndarray) -> np.ndarray:
    L8 = np.ascontiguousarray(L8, dtype=np.uint8)
    out = np.empty(L8.shape, np.uint8)
    _load().oracle_label_pixels(_p(L8), L8.size, _p(np.ascontiguousarray(bin_label, np.int32)), _p(out))
    return out


def _map_op(name, m):
    m = np.ascontiguousarray(m, dtype=np.uint8)
    H, W = m.shape
    out = np.empty_like(m)
    getattr(_load(), name)(_p(m), W, H, _p(out))
    return out


def label_open_close(lab):
    return _map_op("oracle_label_open_close", lab)


def erode3(m):
    return _map_op("oracle_erode3", m)


def dilate3(m):
    return _map_op("oracle_dilate3", m)


def boundary(lab):
    return _map_op("oracle_boundary", lab)


def fill(B):
    return _map_op("oracle_fill", B)


def remove(B):
    return _map_op("oracle_remove", B)


def components(B: np.ndarray):
    B = np.ascontiguousarray(B, dtype=np.uint8)
    H, W = B.shape
    comp = np.empty((H, W), np.int32)
    sizes = np.empty(H * W + 1, np.int64)
    nc = _load().oracle_components(_p(B), W, H, _p(comp), _p(sizes))
    return comp, sizes[:nc].copy()


def cc_filter(B: np.ndarray, mode: int = 0, min_size: int = 50, drop_frac: float = 0.04):
    B = np.ascontiguousarray(B, dtype=np.uint8)
    H, W = B.shape
    out = np.empty_like(B)
    _load().oracle_cc_filter(_p(B), W, H, mode, min_size, drop_frac, _p(out))
    return out


def boundaries(img: np.ndarray, K: int = 4, mode: int = 0, min_cc: int = 50, frac: float = -1.0,
               seed: int = 0, return_map: bool = False):
    """Ascending uint32 list of boundary pixels from the full front end."""
    img, W, H, C, pitch = _img(img)
    cap = W * H
    out = np.empty(cap, np.uint32)
    rmap = np.empty((H, W), np.uint8)
    n = _load().oracle_boundaries(_p(img), W, H, C, pitch, K, mode, min_cc, float(frac),
                                  seed & (2**64 - 1), _p(out), cap, _p(rmap))
    if n < 0:
        raise ValueError("oracle_boundaries failed")
    lst = out[:n].copy()
    return (lst, rmap) if return_map else lst


def fraction_select(refined: np.ndarray, frac: float, seed: int = 0) -> np.ndarray:
    """Border columns plus refined pixels (frac < 0), or exactly round(frac*W*H)
    pixels by the fixed ranking; ascending uint32 raster indices."""
    refined = np.ascontiguousarray(refined, dtype=np.uint8)
    H, W = refined.shape
    out = np.empty(W * H, np.uint32)
    n = _load().oracle_fraction_select(_p(refined), W, H, float(frac), seed & (2**64 - 1), _p(out), W * H)
    if n < 0:
        raise ValueError("oracle_fraction_select failed")
    return out[:n].copy()


def sad(left: np.ndarray, right: np.ndarray, idx: np.ndarray, block: int, dmax: int,
        threads: int | None = None):
    """Brute-force SAD-WTA at the listed pixels. Returns (disp u8, cost u32, status)."""
    left, W, H, C, pitch = _img(left)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    assert right.shape == left.shape
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    n = idx.size
    disp = np.empty(n, np.uint8)
    cost = np.empty(n, np.uint32)
    if threads is None:
        threads = os.cpu_count() or 1
    rc = _load().oracle_sad(_p(left), _p(right), W, H, C, pitch, _p(idx), n, block, dmax,
                            _p(disp), _p(cost), threads)
    if rc == 1:
        raise ValueError("invalid arguments")
    return disp, cost, rc


def sad_sat(left, right, idx, block, dmax):
    """Same SAD-WTA by summed-area tables (independent algorithm)."""
    left, W, H, C, pitch = _img(left)
    right = np.ascontiguousarray(right, dtype=np.uint8)
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    n = idx.size
    disp = np.empty(n, np.uint8)
    cost = np.empty(n, np.uint32)
    rc = _load().oracle_sad_sat(_p(left), _p(right), W, H, C, pitch, _p(idx), n, block, dmax,
                                _p(disp), _p(cost))
    if rc == 1:
        raise ValueError("invalid arguments")
    return disp, cost, rc


def reconstruct(idx, disp, W: int, H: int, threshold: int) -> np.ndarray:
    idx = np.ascontiguousarray(idx, dtype=np.uint32)
    disp = np.ascontiguousarray(disp, dtype=np.uint8)
    out = np.empty((H, W), np.uint8)
    _load().oracle_reconstruct(_p(idx), _p(disp), idx.size, W, H, threshold, _p(out))
    return out


def blur(img: np.ndarray, depth: np.ndarray, ranges, sigma: float) -> np.ndarray:
    img, W, H, C, pitch = _img(img)
    depth = np.ascontiguousarray(depth, dtype=np.uint8)
    rg = np.ascontiguousarray(np.asarray(ranges, dtype=np.int32).reshape(-1))
    out = np.empty((H, W, C) if C > 1 else (H, W), np.float32)
    _load().oracle_blur(_p(img), W, H, C, pitch, _p(depth), _p(rg), rg.size // 2, float(sigma), _p(out))
    return out
