"""Boundary-pixel SAD stereo disparity on AMD Instinct MI355X (gfx950).

This is a thin binding over ``libsbs.so`` (the C-ABI in ``include/sbs.h``) and
does argument marshalling only. Every step of the computation runs in the HIP
kernels under ``csrc/``. PyTorch supplies device memory and streams. There is no
CPU fallback: if the library is missing or no gfx950 device is present, calls
raise.

The operation (arXiv 2001.07809, Sec. III "Disparity Measurement of Boundary
Pixels", winner-takes-all of Sec. II): for each listed pixel, the disparity d
in [0, dmax] minimising the block x block sum of absolute differences between
the left window at x and the right window at x - d on the same rows
(replicate padding, ties to the smaller d).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_CSRC = os.path.join(_HERE, "csrc")
_SO = os.path.join(_HERE, "libsbs.so")
_lib = None

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]

SBS_OK = 0
STATUS = {0: "SBS_OK", 1: "SBS_ERR_INVALID_ARG", 2: "SBS_ERR_UNSUPPORTED", 3: "SBS_ERR_WORKSPACE",
          4: "SBS_ERR_HIP", 5: "SBS_ERR_INDEX_RANGE"}


class SbsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def build() -> str:
    """Compile libsbs.so for gfx950 (always recompiles)."""
    srcs = [os.path.join(_CSRC, "sbs_kernels.hip"), os.path.join(_CSRC, "sbs_api.hip"),
            os.path.join(_CSRC, "sbs_post.hip"), os.path.join(_CSRC, "sbs_front.hip"),
            os.path.join(_CSRC, "sbs_noalloc.hip"), os.path.join(_CSRC, "sbs_probe.hip")]
    cmd = [HIPCC, *HIP_FLAGS, *srcs, "-o", _SO + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stderr[-4000:])
    os.replace(_SO + ".tmp", _SO)
    return _SO


class Frame(ctypes.Structure):
    """sbs_frame (host descriptor of one frame)."""
    _fields_ = [
        ("left", ctypes.c_void_p), ("right", ctypes.c_void_p),
        ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("C", ctypes.c_int32),
        ("pitch_bytes", ctypes.c_int64),
        ("boundary_idx", ctypes.c_void_p), ("n", ctypes.c_int64),
        ("block", ctypes.c_int32), ("dmax", ctypes.c_int32),
        ("out_disp", ctypes.c_void_p), ("out_cost", ctypes.c_void_p),
    ]


class Plan(ctypes.Structure):
    _fields_ = [("cols_per_lane", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32)]


def lib():
    """The loaded libsbs.so (built first if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    L = ctypes.CDLL(_SO)
    V, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    FP = ctypes.POINTER(Frame)
    sig = {
        "sbs_sad_disparity": ([V, V, I32, I32, I32, I64, V, I64, I32, I32, V, V, V, SZ, V], ctypes.c_int),
        "sbs_sad_disparity_noalloc": ([V, V, I32, I32, I32, I64, V, I64, I32, I32, V, V, V], ctypes.c_int),
        "sbs_sad_disparity_ref": ([V, V, I32, I32, I32, I64, V, I64, I32, I32, V, V, V], ctypes.c_int),
        "sbs_workspace_bytes": ([FP, I32], SZ),
        "sbs_sad_disparity_batched": ([FP, I32, V, SZ, V], ctypes.c_int),
        "sbs_sad_disparity_per_frame": ([FP, I32, V, SZ, V], ctypes.c_int),
        "sbs_check_indices": ([FP, I32, V, V], ctypes.c_int),
        "sbs_tune": ([FP, I32, ctypes.c_char_p], ctypes.c_int),
        "sbs_load_tuning": ([ctypes.c_char_p], ctypes.c_int),
        "sbs_last_error": ([], ctypes.c_char_p),
        "sbs_abi_version": ([], ctypes.c_int),
        "sbs_set_plan": ([ctypes.POINTER(Plan)], ctypes.c_int),
        "sbs_get_plan": ([FP, ctypes.POINTER(Plan)], ctypes.c_int),
        "sbs_get_plan_batched": ([FP, I32, ctypes.POINTER(Plan)], ctypes.c_int),
        "sbs_kernel_timing": ([I32], ctypes.c_int),
        "sbs_reconstruct_workspace_bytes": ([I32, I32], SZ),
        "sbs_reconstruct": ([V, V, I64, I32, I32, I32, V, V, SZ, V], ctypes.c_int),
        "sbs_selective_blur_workspace_bytes": ([I32, I32, I32], SZ),
        "sbs_selective_blur": ([V, I32, I32, I32, I64, V, V, I32, ctypes.c_float, V, V, SZ, V], ctypes.c_int),
        "sbs_kernel_times": ([ctypes.POINTER(ctypes.c_float), I32], I32),
        "sbs_lightness": ([V, I32, I32, I32, I64, V, V], ctypes.c_int),
        "sbs_boundaries_workspace_bytes": ([I32, I32], SZ),
        "sbs_probe_sad_rate": ([I32, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                               ctypes.c_int),
        "sbs_boundaries": ([V, I32, I32, I32, I64, I32, I32, I32, ctypes.c_double, ctypes.c_uint64, V, V, V, V, V,
                            SZ, V], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(status: int):
    if status != SBS_OK:
        raise SbsError(status, lib().sbs_last_error().decode())


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _image_args(img):
    torch = _torch()
    if img.dtype != torch.uint8 or not img.is_cuda:
        raise ValueError("images must be torch.uint8 tensors on the GPU")
    if img.dim() == 2:
        H, W = img.shape
        C = 1
        if img.stride(1) != 1:
            raise ValueError("image columns must be contiguous")
    elif img.dim() == 3 and img.shape[2] == 3:
        H, W, C = img.shape
        if img.stride(2) != 1 or img.stride(1) != 3:
            raise ValueError("RGB images must be HWC with contiguous pixels")
    else:
        raise ValueError("images must be [H, W] or [H, W, 3]")
    return W, H, C, img.stride(0)


def make_frame(left, right, idx, block: int, dmax: int, out_disp, out_cost=None) -> Frame:
    """A host descriptor for the given device tensors (the tensors must outlive its use)."""
    torch = _torch()
    W, H, C, pitch = _image_args(left)
    if right.shape != left.shape or right.stride() != left.stride() or right.dtype != left.dtype:
        raise ValueError("left and right must have the same shape and layout")
    if idx.dtype not in (torch.int32, torch.uint32) or not idx.is_contiguous():
        raise ValueError("idx must be a contiguous int32 tensor")
    n = idx.numel()
    if out_disp.numel() < n or out_disp.dtype != torch.uint8:
        raise ValueError("out_disp must be uint8 with >= n elements")
    if out_cost is not None and (out_cost.numel() < n or out_cost.dtype not in (torch.int32, torch.uint32)):
        raise ValueError("out_cost must be int32/uint32 with >= n elements")
    return Frame(left.data_ptr(), right.data_ptr(), W, H, C, pitch, idx.data_ptr(), n, block, dmax,
                 out_disp.data_ptr(), None if out_cost is None else out_cost.data_ptr())


def sad_disparity(left, right, idx, block: int, dmax: int, out=None, cost=None, stream=None,
                  workspace=None, with_cost: bool = True):
    """Disparity (uint8) and cost (int32 holding u32) at the listed pixels.

    left/right: torch.uint8 [H, W] or [H, W, 3] on the GPU; idx: int32 [n] of
    raster indices y*W + x. Returns (disp, cost); cost is None if with_cost is
    False and no cost tensor was given.
    """
    torch = _torch()
    n = idx.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=left.device)
    if cost is None and with_cost:
        cost = torch.empty(n, dtype=torch.int32, device=left.device)
    f = make_frame(left, right, idx, block, dmax, out, cost)
    ws_ptr, ws_bytes = (None, 0)
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    _check(lib().sbs_sad_disparity(f.left, f.right, f.W, f.H, f.C, f.pitch_bytes, f.boundary_idx, f.n,
                                   f.block, f.dmax, f.out_disp, f.out_cost, ws_ptr, ws_bytes,
                                   _stream_handle(stream)))
    return out, cost


def sad_disparity_noalloc(left, right, idx, block: int, dmax: int, out=None, cost=None, stream=None):
    """sad_disparity in the library's fixed device scratch (no allocation by
    the library; ``out``/``cost`` are allocated here when not given)."""
    torch = _torch()
    n = idx.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=left.device)
    if cost is None:
        cost = torch.empty(n, dtype=torch.int32, device=left.device)
    f = make_frame(left, right, idx, block, dmax, out, cost)
    _check(lib().sbs_sad_disparity_noalloc(f.left, f.right, f.W, f.H, f.C, f.pitch_bytes, f.boundary_idx, f.n,
                                           f.block, f.dmax, f.out_disp, f.out_cost, _stream_handle(stream)))
    return out, cost


SCRATCH_BYTES = 160 << 20


def sad_disparity_ref(left, right, idx, block: int, dmax: int, out=None, cost=None, stream=None):
    """The brute-force reference kernel (separate code path), same results."""
    torch = _torch()
    n = idx.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.uint8, device=left.device)
    if cost is None:
        cost = torch.empty(n, dtype=torch.int32, device=left.device)
    f = make_frame(left, right, idx, block, dmax, out, cost)
    _check(lib().sbs_sad_disparity_ref(f.left, f.right, f.W, f.H, f.C, f.pitch_bytes, f.boundary_idx, f.n,
                                       f.block, f.dmax, f.out_disp, f.out_cost, _stream_handle(stream)))
    return out, cost


def probe_sad_rate(blocks: int = 8192, trips: int = 2000) -> dict:
    """v_sad_u8 lane operations per second with every wavefront slot busy
    (sbs_probe_sad_rate; synchronous)."""
    rate, ms = ctypes.c_double(), ctypes.c_double()
    _check(lib().sbs_probe_sad_rate(blocks, trips, ctypes.byref(rate), ctypes.byref(ms)))
    return {"lane_ops_per_s": rate.value, "ms": ms.value, "blocks": blocks, "trips": trips}


def workspace_bytes(frames) -> int:
    arr = (Frame * len(frames))(*frames)
    return int(lib().sbs_workspace_bytes(arr, len(frames)))


def check_indices(workspace=None, stream=None) -> int:
    """Reads and clears the device error word; returns the status (0 or 5)."""
    ws = None if workspace is None else ctypes.c_void_p(workspace.data_ptr())
    return int(lib().sbs_check_indices(None, 0, ws, _stream_handle(stream)))


def set_plan(cols_per_lane=0, chunk=0, tile_rows=0, waves_per_cu=0):
    p = Plan(cols_per_lane, chunk, tile_rows, waves_per_cu)
    _check(lib().sbs_set_plan(ctypes.byref(p)))


def get_plan(frame: Frame) -> dict:
    p = Plan()
    _check(lib().sbs_get_plan(ctypes.byref(frame), ctypes.byref(p)))
    return {"cols_per_lane": p.cols_per_lane, "chunk": p.chunk, "tile_rows": p.tile_rows,
            "waves_per_cu": p.waves_per_cu}


def kernel_timing(enable: bool):
    """Record HIP events around every tile-kernel launch while enabled."""
    _check(lib().sbs_kernel_timing(1 if enable else 0))


def kernel_times() -> list:
    """Durations (ms) of the tile-kernel launches recorded since the last call."""
    cap = 1 << 16
    buf = (ctypes.c_float * cap)()
    n = int(lib().sbs_kernel_times(buf, cap))
    return [buf[i] for i in range(min(n, cap))]


def tune(frames, cache_path: str | None = None):
    arr = (Frame * len(frames))(*frames)
    _check(lib().sbs_tune(arr, len(frames), None if cache_path is None else cache_path.encode()))


def load_tuning(cache_path: str):
    _check(lib().sbs_load_tuning(cache_path.encode()))


def reconstruct(idx, disp, W: int, H: int, threshold: int, stream=None):
    """Dense u8 disparity map [H, W] from listed pixels (Algorithms 1 and 2)."""
    torch = _torch()
    dev = idx.device
    out = torch.empty((H, W), dtype=torch.uint8, device=dev)
    nb = int(lib().sbs_reconstruct_workspace_bytes(W, H))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    _check(lib().sbs_reconstruct(idx.data_ptr(), disp.data_ptr(), idx.numel(), W, H, threshold, out.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream_handle(stream)))
    return out


def selective_blur(img, depth, ranges, sigma: float, stream=None):
    """Float32 HWC image with pixels outside the depth ranges blurred (Eq. 1-2)."""
    torch = _torch()
    W, H, C, pitch = _image_args(img)
    rg = (ctypes.c_int32 * max(2 * len(ranges), 2))(*[int(v) for pr in ranges for v in pr])
    out = torch.empty(img.shape, dtype=torch.float32, device=img.device)
    nb = int(lib().sbs_selective_blur_workspace_bytes(W, H, C))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=img.device)
    _check(lib().sbs_selective_blur(img.data_ptr(), W, H, C, pitch, depth.data_ptr(), rg, len(ranges),
                                    float(sigma), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                    _stream_handle(stream)))
    return out


def lightness(img, stream=None):
    """u8 lightness [H, W] of a device image (gray passes through)."""
    torch = _torch()
    W, H, C, pitch = _image_args(img)
    out = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    _check(lib().sbs_lightness(img.data_ptr(), W, H, C, pitch, out.data_ptr(), _stream_handle(stream)))
    return out


def boundaries(img, K: int = 4, mode: int = 0, min_cc: int = 50, frac: float = -1.0, seed: int = 0,
               with_maps: bool = False, stream=None):
    """Ascending int32 device list of refined boundary pixels (plus border
    columns) of a device image; with ``frac >= 0`` exactly round(frac*W*H)
    pixels by the fixed ranking. With ``with_maps`` also returns the kept
    boundary map and the label image [H, W] u8."""
    torch = _torch()
    W, H, C, pitch = _image_args(img)
    dev = img.device
    out = torch.empty(W * H, dtype=torch.int32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    refined = torch.empty((H, W), dtype=torch.uint8, device=dev) if with_maps else None
    labels = torch.empty((H, W), dtype=torch.uint8, device=dev) if with_maps else None
    nb = int(lib().sbs_boundaries_workspace_bytes(W, H))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=dev)
    _check(lib().sbs_boundaries(img.data_ptr(), W, H, C, pitch, K, mode, min_cc, float(frac), seed & (2**64 - 1),
                                out.data_ptr(), count.data_ptr(),
                                None if refined is None else refined.data_ptr(),
                                None if labels is None else labels.data_ptr(), ws.data_ptr(), ws.numel(),
                                _stream_handle(stream)))
    n = int(count.item())
    lst = out[:n]
    return (lst, refined, labels) if with_maps else lst


class BatchRunner:
    """Many frames through one persistent launch.

    ``frames`` is a list of (left, right, idx, block, dmax) device-tensor
    tuples. Outputs are allocated here (``disp[i]``, ``cost[i]``). The
    workspace is one device tensor sized by sbs_workspace_bytes. ``run``
    enqueues the batched path; ``run_per_frame`` enqueues the same work as
    separate launches per frame (for comparison). Both are capture safe.
    """

    def __init__(self, frames, with_cost: bool = True, device=None):
        torch = _torch()
        self.inputs = list(frames)
        dev = device or (self.inputs[0][0].device if self.inputs else torch.device("cuda"))
        self.disp, self.cost, descs = [], [], []
        for (l, r, idx, block, dmax) in self.inputs:
            n = idx.numel()
            d = torch.empty(n, dtype=torch.uint8, device=dev)
            c = torch.empty(n, dtype=torch.int32, device=dev) if with_cost else None
            self.disp.append(d)
            self.cost.append(c)
            descs.append(make_frame(l, r, idx, block, dmax, d, c))
        self.nframes = len(descs)
        self.desc = (Frame * max(self.nframes, 1))(*descs)
        nbytes = int(lib().sbs_workspace_bytes(self.desc, self.nframes))
        if self.nframes and nbytes == 0:
            raise SbsError(1, lib().sbs_last_error().decode())
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self.workspace[:256].zero_()

    def _ws(self):
        return ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel()

    def run(self, stream=None):
        p, b = self._ws()
        _check(lib().sbs_sad_disparity_batched(self.desc, self.nframes, p, b, _stream_handle(stream)))

    def run_per_frame(self, stream=None):
        p, b = self._ws()
        _check(lib().sbs_sad_disparity_per_frame(self.desc, self.nframes, p, b, _stream_handle(stream)))

    def check_indices(self, stream=None) -> int:
        return check_indices(self.workspace, stream)

    def plan(self) -> dict:
        """The plan a batched call on these frames runs with."""
        p = Plan()
        _check(lib().sbs_get_plan_batched(self.desc, self.nframes, ctypes.byref(p)))
        return {"cols_per_lane": p.cols_per_lane, "chunk": p.chunk, "tile_rows": p.tile_rows,
                "waves_per_cu": p.waves_per_cu}

    def tune(self, cache_path: str | None = None):
        """Autotune the plan of a batched call on these frames (sbs_tune)."""
        _check(lib().sbs_tune(self.desc, self.nframes, None if cache_path is None else cache_path.encode()))
