"""Continuous-batching render server over a device-resident surfel set (novel-view renders of mixed
resolutions; the rendering FPS workloads of CityGaussianV2 Sec. 5).

Requests arrive at any time (``submit``).  The scheduler admits the head of the queue as soon as a
slot is free *and* the request's memory estimate fits the arena budget, launches its
project -> bin_sort -> render_fwd on the slot's own stream (all streams at default priority), and
keeps admitting while earlier requests are still on the GPU, so the work of different requests
overlaps on the device.  Completion is observed with events; a request whose intersections
overflowed its bins is re-admitted with the reported size.  Latency = completion - arrival.

Results are device tensors owned by the request (rgb [3,H,W], depth [H,W], normal [3,H,W]); the
render is deterministic, so a request's result is the same alone and in any mix.
"""
from __future__ import annotations

import collections
import time
from typing import Deque, List, Optional

import torch

from . import _lib, raster


class Request:
    __slots__ = ("rid", "cam", "arrival", "admitted", "done_t", "result", "capacity", "est_bytes", "tries",
                 "error", "_event", "_slot")

    def __init__(self, rid: int, cam, arrival: float, capacity: int):
        self.rid, self.cam, self.arrival = rid, cam, arrival
        self.admitted = self.done_t = None
        self.result = None
        self.capacity = capacity
        self.est_bytes = 0
        self.tries = 0
        self.error = None
        self._event = None
        self._slot = None

    @property
    def done(self) -> bool:
        return self.done_t is not None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_t is None else self.done_t - self.arrival


class _Slot:
    """Per-slot projection buffers (n surfels, one view) and stream; bins/images per request."""

    def __init__(self, n: int, max_w: int, max_h: int, device):
        self.stream = torch.cuda.Stream(device=device)  # default priority
        with torch.cuda.stream(self.stream):
            self.eng = raster.Engine(n, max_w, max_h, 1, capacity=1, device=device, backward=False)
        # status and needed count, copied to pinned host memory on the slot's stream
        self.host = torch.zeros(2, dtype=torch.int64, pin_memory=True)
        self.req: Optional[Request] = None


class Server:
    def __init__(self, params: raster.Params, max_slots: int = 4, arena_bytes: int = 8 << 30,
                 max_width: int = 3840, max_height: int = 2160, intersections_per_pixel: float = 2.0,
                 keep_results: bool = True, device="cuda"):
        self.params = params
        # False: a finished request's images are released at once (load generators that only time)
        self.keep_results = keep_results
        self.n = params.n
        self.max_w, self.max_h = max_width, max_height
        self.arena_bytes = int(arena_bytes)
        self.arena_used = 0
        # intersections per pixel used to size a request's bins; raised to the largest ratio any
        # finished request reported (x 1.1), so overflow re-admissions die out after a few requests
        self.ipp = float(intersections_per_pixel)
        self.slots = [_Slot(self.n, max_width, max_height, device) for _ in range(max_slots)]
        self.queue: Deque[Request] = collections.deque()
        self.finished: List[Request] = []
        self._next = 0
        self.device = device

    # ---- client side -------------------------------------------------------------------------
    def submit(self, cam, arrival: Optional[float] = None) -> Request:
        if cam.width > self.max_w or cam.height > self.max_h:
            raise ValueError("resolution above the server's maximum")
        r = Request(self._next, cam, time.perf_counter() if arrival is None else arrival, 0)
        self._next += 1
        self.queue.append(r)
        return r

    # ---- scheduler -----------------------------------------------------------------------------
    def _estimate(self, r: Request) -> int:
        px = r.cam.width * r.cam.height
        L = _lib.lib()
        ws = L.cgv2_bin_sort_workspace(r.capacity, 1, ((r.cam.width + 15) // 16) * ((r.cam.height + 15) // 16), self.n)
        return ws + 4 * r.capacity + 28 * px  # workspace, ids, rgb + depth + normal copies

    def _launch(self, slot: _Slot, r: Request):
        eng = slot.eng
        with torch.cuda.stream(slot.stream):
            eng.set_capacity(r.capacity)
            eng.status.zero_()
            cams = eng.cams([r.cam], exact=False)
            eng.forward(self.params, cams)
            W, H = r.cam.width, r.cam.height
            r.result = dict(rgb=eng.image("rgb", W, H).clone(), depth=eng.image("depth", W, H).clone(),
                            normal=eng.image("normal", W, H).clone())
            slot.host[0:1].copy_(eng.status, non_blocking=True)
            slot.host[1:2].copy_(eng.needed, non_blocking=True)
            r._event = torch.cuda.Event()
            r._event.record(slot.stream)
        r._slot = slot
        slot.req = r

    def poll(self) -> int:
        """Retire finished requests, then admit as many queued ones as slots and memory allow.
        Returns the number of requests still queued or running."""
        now = time.perf_counter()
        for slot in self.slots:
            r = slot.req
            if r is None or not r._event.query():
                continue
            over = int(slot.host[0]) != 0
            need = int(slot.host[1])
            slot.req = None
            self.arena_used -= r.est_bytes
            self.ipp = max(self.ipp, 1.1 * need / (r.cam.width * r.cam.height))
            if over:
                # bins too small: re-admit first with the reported size
                r.capacity = int(need * 1.05) + 1024
                r.result = None
                r.tries += 1
                self.queue.appendleft(r)
                continue
            r.done_t = now
            if not self.keep_results:
                r.result = None
            self.finished.append(r)
        for slot in self.slots:
            if slot.req is not None or not self.queue:
                continue
            r = self.queue[0]
            if r.tries == 0:
                r.capacity = int(self.ipp * r.cam.width * r.cam.height) + 4096
            est = self._estimate(r)
            if est > self.arena_bytes:
                self.queue.popleft()
                r.error = "request exceeds the arena"
                r.done_t = now
                self.finished.append(r)
                continue
            if self.arena_used + est > self.arena_bytes:
                break  # wait for memory (FIFO: no overtaking)
            self.queue.popleft()
            r.est_bytes = est
            r.admitted = time.perf_counter()
            self.arena_used += est
            self._launch(slot, r)
        return len(self.queue) + sum(s.req is not None for s in self.slots)

    def drain(self):
        while self.poll():
            time.sleep(50e-6)

    def render_alone(self, cam):
        """One request through an otherwise idle server (reference for the alone-vs-mix check)."""
        r = self.submit(cam)
        self.drain()
        return r


def run_trace(server: Server, cams, arrivals, spin: float = 50e-6):
    """Open-loop replay: request k is submitted at arrivals[k] seconds after the start."""
    t0 = time.perf_counter()
    reqs = []
    k = 0
    while k < len(arrivals) or server.poll():
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k] <= now:
            reqs.append(server.submit(cams[k], arrival=t0 + arrivals[k]))
            k += 1
        server.poll()
        time.sleep(spin)
    return reqs, time.perf_counter() - t0
