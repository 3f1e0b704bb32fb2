"""Serving loop with continuous batching for boundary-pixel SAD disparity.

Requests are frames with their boundary lists (device tensors; a request's
inputs stay resident in HBM from arrival to completion). The server:

* admits waiting requests in arrival order while the HBM footprint of the
  work in flight stays within a byte budget and a batch slot is free. The
  footprint of a request is its workspace share plus its outputs;
* launches each admitted group as ONE persistent batched call
  (``sbs_sad_disparity_batched``). Up to ``max_inflight`` batches run at once
  on separate HIP streams, so requests that arrive while others are on the GPU
  are admitted as soon as a slot and memory free up, and their work overlaps
  on the device;
* completes a request when its batch's HIP event has fired, and records its
  latency (completion minus arrival).

A request may also come as a raw frame without a list (``idx=None``, with a
boundary fraction ``frac``): the server then runs the front end first
(lightness, histogram K-means, refinement, components, fraction control) into
a list of exactly round(frac * W * H) pixels, whose length is known on the
host, so nothing waits for the device. A batch's raw frames are dealt over
``fe_lanes`` streams (its own and side streams shared by all batches), each
with one front-end workspace for its frames in turn, so the many short
front-end kernels of small frames overlap; the batch's stream waits for all
lanes before the disparity search. The workspaces count against the budget.

Each request's result depends only on its own frame: it is the same alone and
in any mix (the GPU tests check this bit for bit).
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import paper_2001_07809_amd as sbs


@dataclass
class Request:
    rid: int
    left: object            # torch.uint8 [H, W] or [H, W, 3] on the GPU
    right: object
    idx: object             # torch.int32 [n] on the GPU, or None: list from the front end
    block: int
    dmax: int
    arrival: float = 0.0    # seconds on the server clock
    klass: str = ""
    frac: float = 0.18      # raw frames: boundary fraction of the list the front end makes
    K: int = 4              # raw frames: front-end clusters
    seed: int = 0           # raw frames: fraction-control seed
    disp: object = None
    cost: object = None
    t_admit: float = -1.0
    t_done: float = -1.0
    footprint: int = 0


@dataclass
class _Batch:
    reqs: list
    workspace: object
    desc: object
    event: object
    stream: object
    nbytes: int
    keep: list = field(default_factory=list)   # buffers the batch's kernels use until its event fires


class BudgetError(RuntimeError):
    pass


class Server:
    def __init__(self, budget_bytes: int, max_inflight: int = 2, max_batch: int = 64, device=None,
                 with_cost: bool = True, fe_lanes: int = 3):
        import torch
        self.torch = torch
        self.device = device or torch.device("cuda")
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.with_cost = with_cost
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        # front-end side streams (default priority), shared by all batches
        self.fe_side = [torch.cuda.Stream(device=self.device) for _ in range(max(0, fe_lanes - 1))]
        self._next_stream = 0
        self.waiting: list[Request] = []
        self.inflight: list[_Batch] = []
        self.done: list[Request] = []
        self.in_use = 0
        self.peak_in_use = 0
        self.batches = 0
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- footprint ---------------------------------------------------------
    def _frame(self, r: Request, disp, cost):
        return sbs.make_frame(r.left, r.right, r.idx, r.block, r.dmax, disp, cost)

    def list_length(self, r: Request) -> int:
        if r.idx is not None:
            return r.idx.numel()
        import math
        N = r.left.shape[0] * r.left.shape[1]
        return min(N, int(math.floor(r.frac * N + 0.5)))   # the front end's round-half-away length

    def footprint(self, r: Request) -> int:
        n = self.list_length(r)
        W, H, C, pitch = sbs._image_args(r.left)
        f = sbs.Frame(r.left.data_ptr(), r.right.data_ptr(), W, H, C, pitch, 1, max(n, 1), r.block, r.dmax, 1, None)
        ws = sbs.workspace_bytes([f])
        if ws == 0:
            raise ValueError(f"request {r.rid}: invalid frame")
        extra = 0
        if r.idx is None:
            # its list, plus (conservatively) a whole front-end workspace
            extra = 4 * n + int(sbs.lib().sbs_boundaries_workspace_bytes(W, H))
        return ws + n * (5 if self.with_cost else 1) + extra + 4096

    def submit(self, r: Request):
        r.footprint = self.footprint(r)
        if r.footprint > self.budget:
            raise BudgetError(f"request {r.rid} needs {r.footprint} bytes, budget is {self.budget}")
        self.waiting.append(r)

    # -- engine ------------------------------------------------------------
    def poll(self):
        still = []
        for b in self.inflight:
            if b.event.query():
                t = self.now()
                for r in b.reqs:
                    r.t_done = t
                    self.done.append(r)
                self.in_use -= b.nbytes
            else:
                still.append(b)
        self.inflight = still

    def launch(self) -> bool:
        """Admit what fits and launch one batch. Returns True if a batch was launched."""
        torch = self.torch
        if not self.waiting or len(self.inflight) >= self.max_inflight:
            return False
        free = self.budget - self.in_use
        take, total = [], 0
        for r in self.waiting:
            if len(take) >= self.max_batch or total + r.footprint > free:
                break
            take.append(r)
            total += r.footprint
        if not take:
            return False
        self.waiting = self.waiting[len(take):]
        t = self.now()
        stream = self.streams[self._next_stream]
        self._next_stream = (self._next_stream + 1) % len(self.streams)
        stream.wait_stream(torch.cuda.current_stream())   # inputs and outputs were made on the caller's stream
        frames = []
        keep = []
        raw = [r for r in take if r.idx is None]
        if raw:
            # lists of the raw frames, dealt over the front-end lanes; each lane
            # starts once the batch's stream has its inputs, and the batch's
            # stream waits for every lane before the search
            lanes = [stream] + self.fe_side[:len(raw) - 1]
            ready = torch.cuda.Event()
            ready.record(stream)
            for li, lane in enumerate(lanes):
                mine = raw[li::len(lanes)]
                if lane is not stream:
                    lane.wait_event(ready)
                with torch.cuda.stream(lane):
                    fw = max(int(sbs.lib().sbs_boundaries_workspace_bytes(*sbs._image_args(r.left)[:2])) for r in mine)
                    fws = torch.empty(max(fw, 256), dtype=torch.uint8, device=self.device)
                    cnt = torch.empty(1, dtype=torch.int64, device=self.device)
                    keep += [fws, cnt]
                    for r in mine:
                        W, H, C, pitch = sbs._image_args(r.left)
                        r.idx = torch.empty(self.list_length(r), dtype=torch.int32, device=self.device)
                        if lane is not stream:
                            r.idx.record_stream(stream)   # read by the search on the batch's stream
                        if r.idx.numel() == 0:
                            continue
                        sbs._check(sbs.lib().sbs_boundaries(r.left.data_ptr(), W, H, C, pitch, r.K, 0, 50,
                                                            float(r.frac), r.seed & (2**64 - 1), r.idx.data_ptr(),
                                                            cnt.data_ptr(), None, None, fws.data_ptr(), fws.numel(),
                                                            ctypes.c_void_p(lane.cuda_stream)))
                if lane is not stream:
                    done = torch.cuda.Event()
                    done.record(lane)
                    stream.wait_event(done)
        with torch.cuda.stream(stream):
            for r in take:
                n = r.idx.numel()
                r.disp = torch.empty(n, dtype=torch.uint8, device=self.device)
                r.cost = torch.empty(n, dtype=torch.int32, device=self.device) if self.with_cost else None
                r.t_admit = t
                frames.append(self._frame(r, r.disp, r.cost))
        desc = (sbs.Frame * len(frames))(*frames)
        nbytes = int(sbs.lib().sbs_workspace_bytes(desc, len(frames)))
        with torch.cuda.stream(stream):
            ws = torch.empty(max(nbytes, 1024), dtype=torch.uint8, device=self.device)
            ws[:1024].zero_()
            sbs._check(sbs.lib().sbs_sad_disparity_batched(desc, len(frames), ctypes.c_void_p(ws.data_ptr()),
                                                           ws.numel(), ctypes.c_void_p(stream.cuda_stream)))
            ev = torch.cuda.Event()
            ev.record(stream)
        self.in_use += total
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        self.inflight.append(_Batch(take, ws, desc, ev, stream, total, keep))
        self.batches += 1
        return True

    def drain(self):
        while self.waiting or self.inflight:
            self.poll()
            self.launch()

    def run_trace(self, requests: list[Request]) -> dict:
        """Replays requests at their arrival times (seconds after start) and returns latency stats."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = time.perf_counter()
        i = 0
        while i < len(pending) or self.waiting or self.inflight:
            t = self.now()
            while i < len(pending) and pending[i].arrival <= t:
                self.submit(pending[i])
                i += 1
            self.poll()
            launched = self.launch()
            if not launched and i < len(pending) and not self.inflight and not self.waiting:
                # idle until the next arrival
                dt = pending[i].arrival - self.now()
                if dt > 0:
                    time.sleep(min(dt, 0.0005))
        return self.stats(requests)

    def stats(self, requests: list[Request]) -> dict:
        import numpy as np
        lat = np.array([r.t_done - r.arrival for r in requests])
        span = max(r.t_done for r in requests) - min(r.arrival for r in requests)
        out = {
            "requests": len(requests),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "frames_per_s": len(requests) / span if span > 0 else float("inf"),
            "batches": self.batches,
            "peak_bytes_in_flight": self.peak_in_use,
            "budget_bytes": self.budget,
        }
        by = {}
        for k in sorted({r.klass for r in requests}):
            lk = np.array([r.t_done - r.arrival for r in requests if r.klass == k])
            by[k] = {"n": int(lk.size), "p50_ms": float(np.percentile(lk, 50) * 1e3),
                     "p99_ms": float(np.percentile(lk, 99) * 1e3)}
        out["by_class"] = by
        return out
