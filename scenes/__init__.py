"""Seeded synthetic stereo scenes (the input generator).

Shared by the tests, the benchmark and the oracle's checks. It holds none of
the disparity method's arithmetic. The C++ source is ``scenes.cpp``. ``build()``
compiles it to ``libscenes.so`` in this folder.

Workload presets stand in for the paper's inputs. None of the paper's images
are used:
  * ``tsukuba_gray``: 384x288 gray, 6 regions, disparity 0..15
    (the shape and range of the Middlebury Tsukuba pair), block 15, dmax 15.
  * ``middlebury_rgb``: 1390x1110 RGB, 20 regions, disparity 0..63, one
    0..8 px ramp, Gaussian-smoothed texture, additive noise sigma 2,
    block 21, dmax 63.
  * ``tsukuba_paper``, ``middlebury_paper``: the same shapes with 60
    regions of per-region mean lightness (and Gaussian texture), for the
    paper's whole chain: its refinement keeps 16-19% of their pixels, the
    share the paper reports for its Table 3 images.
  * ``uhd_rgb``: 4096x2304 RGB (the paper's video frame size), 40 regions,
    disparity 0..127, per-region mean lightness, block 31, dmax 127.
  * ``uhd_video``: 250 frames of ``uhd_rgb``-like scenes; regions step up to
    4 px per frame and disparities drift by up to 1 per frame; the boundary
    fraction is drawn per frame from [0.12, 0.24].
  * ``serve_*``: the three request classes of the serving mix.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libscenes.so")
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [
        ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("C", ctypes.c_int32),
        ("n_regions", ctypes.c_int32), ("dmax_regions", ctypes.c_int32),
        ("texture", ctypes.c_int32), ("mean_shift", ctypes.c_int32),
        ("ramp", ctypes.c_int32), ("motion", ctypes.c_int32), ("drift", ctypes.c_int32),
        ("noise_sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
    ]


@dataclass(frozen=True)
class SceneSpec:
    W: int
    H: int
    C: int
    n_regions: int
    dmax_regions: int
    texture: int = 0          # 0: 3x3 box smoothed noise, 1: Gaussian sigma 1
    mean_shift: int = 0
    ramp: int = 0
    motion: int = 0
    drift: int = 0
    noise_sigma: float = 0.0
    seed: int = 1
    # matching parameters of the workload
    block: int = 15
    dmax: int = 15
    frac: float = 0.18

    def params(self) -> _Params:
        return _Params(self.W, self.H, self.C, self.n_regions, self.dmax_regions,
                       self.texture, self.mean_shift, self.ramp, self.motion,
                       self.drift, float(self.noise_sigma), self.seed & (2**64 - 1))


PRESETS = {
    "tsukuba_gray": SceneSpec(384, 288, 1, 6, 15, texture=0, seed=101, block=15, dmax=15),
    "middlebury_rgb": SceneSpec(1390, 1110, 3, 20, 63, texture=1, ramp=1, noise_sigma=2.0,
                                seed=102, block=21, dmax=63),
    # the paper chain's inputs at the Tsukuba and Middlebury shapes: more
    # regions with per-region mean lightness, so that K = 10 and the paper's
    # refinement keep 16-19% of the pixels, as the paper reports for its images
    "tsukuba_paper": SceneSpec(384, 288, 1, 60, 15, texture=1, mean_shift=1, seed=101, block=15, dmax=15),
    "middlebury_paper": SceneSpec(1390, 1110, 3, 60, 63, texture=1, mean_shift=1, ramp=1, noise_sigma=2.0,
                                  seed=102, block=21, dmax=63),
    "uhd_rgb": SceneSpec(4096, 2304, 3, 40, 127, texture=0, mean_shift=1, seed=103,
                         block=31, dmax=127),
    "uhd_video": SceneSpec(4096, 2304, 3, 40, 127, texture=0, mean_shift=1, motion=4, drift=1,
                           seed=104, block=31, dmax=127),
    "serve_vga": SceneSpec(640, 480, 3, 10, 31, texture=0, mean_shift=1, seed=105, block=11, dmax=31),
    "serve_fhd": SceneSpec(1920, 1080, 3, 20, 63, texture=0, mean_shift=1, seed=105, block=21, dmax=63),
    "serve_uhd": SceneSpec(4096, 2304, 3, 40, 127, texture=0, mean_shift=1, seed=105, block=31, dmax=127),
}


def build() -> str:
    """Compile libscenes.so (always recompiles)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
           os.path.join(_HERE, "scenes.cpp"), "-o", _SO + ".tmp"]
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
    P = ctypes.POINTER
    lib.sc_frame.argtypes = [P(_Params), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.sc_frame.restype = ctypes.c_int
    lib.sc_contour_list.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p,
                                    ctypes.c_int64]
    lib.sc_contour_list.restype = ctypes.c_int64
    lib.sc_video.argtypes = [P(_Params), ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_int64, ctypes.c_void_p]
    lib.sc_video.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Frame:
    left: np.ndarray    # [H, W] or [H, W, 3] uint8
    right: np.ndarray
    gt: np.ndarray      # [H, W] uint8 owner disparity
    occ: np.ndarray     # [H, W] uint8, 1 = not visible in the right image
    rid: np.ndarray     # [H, W] int16 owning region, -1 = background


def make_frame(spec: SceneSpec, frame: int = 0) -> Frame:
    lib = _load()
    shape = (spec.H, spec.W) if spec.C == 1 else (spec.H, spec.W, spec.C)
    left = np.empty(shape, np.uint8)
    right = np.empty(shape, np.uint8)
    gt = np.empty((spec.H, spec.W), np.uint8)
    occ = np.empty((spec.H, spec.W), np.uint8)
    rid = np.empty((spec.H, spec.W), np.int16)
    p = spec.params()
    rc = lib.sc_frame(ctypes.byref(p), frame, _ptr(left), _ptr(right), _ptr(gt), _ptr(occ), _ptr(rid))
    if rc != 0:
        raise ValueError(f"sc_frame failed for {spec}")
    return Frame(left, right, gt, occ, rid)


def contour_list(rid: np.ndarray, frac: float, seed: int) -> np.ndarray:
    """Ascending uint32 raster indices: border columns, then pixels nearest the region outlines."""
    lib = _load()
    rid = np.ascontiguousarray(rid, dtype=np.int16)
    H, W = rid.shape
    cap = H * W
    out = np.empty(cap, np.uint32)
    n = lib.sc_contour_list(_ptr(rid), W, H, float(frac), seed & (2**64 - 1), _ptr(out), cap)
    if n < 0:
        raise ValueError("sc_contour_list failed")
    return out[:n].copy()


def video_fracs(spec: SceneSpec, frame0: int, nframes: int, lo=0.12, hi=0.24) -> np.ndarray:
    """Per-frame boundary fractions, uniform in [lo, hi], seeded by the scene seed."""
    rng = np.random.Generator(np.random.Philox(key=spec.seed ^ 0x5EED))
    f = rng.uniform(lo, hi, size=frame0 + nframes)
    return f[frame0:].astype(np.float64)


def make_video(spec: SceneSpec, frame0: int, nframes: int, fracs: np.ndarray | None = None,
               with_lists: bool = True):
    """Frames [frame0, frame0+nframes) made in parallel.

    Returns (left [F,H,W,(C)], right, lists (list of uint32 arrays) or None).
    """
    lib = _load()
    shape = (nframes, spec.H, spec.W) if spec.C == 1 else (nframes, spec.H, spec.W, spec.C)
    left = np.empty(shape, np.uint8)
    right = np.empty(shape, np.uint8)
    lists = None
    if with_lists:
        if fracs is None:
            fracs = np.full(nframes, spec.frac)
        fracs = np.ascontiguousarray(fracs, dtype=np.float64)
        cap = int(np.ceil(fracs.max() * spec.W * spec.H)) + 1 if nframes else 1
        buf = np.empty((max(nframes, 1), cap), np.uint32)
        counts = np.zeros(max(nframes, 1), np.int64)
        rc = lib.sc_video(ctypes.byref(spec.params()), frame0, nframes, _ptr(left), _ptr(right),
                          _ptr(fracs), _ptr(buf), cap, _ptr(counts))
        if rc != 0:
            raise ValueError("sc_video failed")
        lists = [buf[i, :counts[i]] for i in range(nframes)]
    else:
        rc = lib.sc_video(ctypes.byref(spec.params()), frame0, nframes, _ptr(left), _ptr(right),
                          None, None, 0, None)
        if rc != 0:
            raise ValueError("sc_video failed")
    return left, right, lists


def scaled(spec: SceneSpec, **kw) -> SceneSpec:
    return replace(spec, **kw)
