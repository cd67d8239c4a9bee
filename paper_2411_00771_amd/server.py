"""Continuous-batching render server over a device-resident surfel set (novel-view renders of mixed
resolutions; the rendering FPS workloads of CityGaussianV2 Sec. 5).

Memory.  The server owns one device budget, ``arena_bytes``.  At start it takes from it each slot's
fixed buffers (projection records, tile ranges and launch order for ``max_batch`` views of n surfels
at the largest resolution) and holds the rest as one preallocated arena.  Every admitted launch takes
one block of the arena, found by first fit: its bins (ids and the bin_sort workspace, sized by the
intersection estimate) and its outputs (rgb, depth and normal of every view).  A launch allocates
nothing: it only binds views of its block.  When it finishes, the results are copied into tensors the
requests own (or dropped, keep_results=False) and the block goes back to the arena.

Scheduling.  Requests arrive at any time (``submit``).  ``poll`` retires finished launches and admits
queued requests while a slot is free and a block fits in the arena: the head of the queue, plus (when
``max_batch`` > 1) the next queued requests of the same resolution, which then render as the views of
one call.  A launch runs project -> bin_sort -> render_fwd on its slot's stream (all streams at the
default priority), so the work of different launches overlaps on the device.  Completion is observed
with events.  A launch whose intersections overflowed its bins is re-admitted first with the reported
size; a request that cannot fit even an empty arena is rejected.  Latency = completion - arrival.

The render is deterministic and a view's render does not depend on the other views of its call, so a
request's result is the same alone and in any mix.
"""
from __future__ import annotations

import collections
import time
from typing import Deque, Dict, List, Optional

import torch

from . import _lib, raster

ALIGN = 256


def _up(x: int) -> int:
    return (int(x) + ALIGN - 1) // ALIGN * ALIGN


class Request:
    __slots__ = ("rid", "cam", "arrival", "admitted", "done_t", "result", "capacity", "tries", "error", "_launch",
                 "_view")

    def __init__(self, rid: int, cam, arrival: float):
        self.rid, self.cam, self.arrival = rid, cam, arrival
        self.admitted = self.done_t = None
        self.result: Optional[Dict[str, torch.Tensor]] = None
        self.capacity = 0  # this request's share of its launch's bins (rect slots)
        self.tries = 0
        self.error = None
        self._launch = None
        self._view = 0

    @property
    def done(self) -> bool:
        return self.done_t is not None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_t is None else self.done_t - self.arrival


class _Arena:
    """First-fit allocator of byte ranges of one preallocated device buffer (256-byte aligned)."""

    def __init__(self, nbytes: int, device):
        self.size = _up(max(nbytes, 0)) if nbytes > 0 else 0
        self.buf = torch.empty(max(self.size, ALIGN), dtype=torch.uint8, device=device)
        self.free = [(0, self.size)] if self.size else []  # sorted, disjoint (offset, length)
        self.used = 0

    def alloc(self, nbytes: int) -> Optional[int]:
        need = _up(max(nbytes, 1))
        for k, (o, ln) in enumerate(self.free):
            if ln >= need:
                self.free[k] = (o + need, ln - need)
                if self.free[k][1] == 0:
                    del self.free[k]
                self.used += need
                return o
        return None

    def release(self, off: int, nbytes: int):
        need = _up(max(nbytes, 1))
        self.used -= need
        self.free.append((off, need))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def view(self, off: int, nbytes: int, dtype, shape):
        t = self.buf[off:off + nbytes].view(dtype)
        return t[: int(torch.Size(shape).numel())].view(shape)


class _Launch:
    __slots__ = ("reqs", "slot", "off", "nbytes", "capacity", "event", "W", "H")


class _Slot:
    """A stream and a render-only engine for up to max_batch views of n surfels (fixed buffers)."""

    def __init__(self, n: int, max_w: int, max_h: int, views: int, device):
        self.stream = torch.cuda.Stream(device=device)  # default priority
        with torch.cuda.stream(self.stream):
            self.eng = raster.Engine(n, max_w, max_h, views, device=device, backward=False, images=False)
        # status and needed count, copied to pinned host memory on the slot's stream
        self.host = torch.zeros(2, dtype=torch.int64, pin_memory=True)
        self.launch: Optional[_Launch] = None

    @staticmethod
    def fixed_bytes(n: int, max_w: int, max_h: int, views: int) -> int:
        """Bytes of a slot's fixed buffers (those of a render-only engine)."""
        tiles = ((max_w + 15) // 16) * ((max_h + 15) // 16)
        vn = max(views * n, 1)
        return (vn * (4 * _lib.REC_FLOATS + 8 + 4 + 1 + 4) + 4 * (views + 1) + 4 * (views * tiles + 1)
                + 4 * views * tiles + 16)


class Server:
    def __init__(self, params: raster.Params, max_slots: int = 4, arena_bytes: int = 8 << 30,
                 max_width: int = 3840, max_height: int = 2160, intersections_per_pixel: float = 2.0,
                 keep_results: bool = True, max_batch: int = 1, device="cuda"):
        self.params = params
        # True: a finished request's result is copied out of the arena into tensors the request owns;
        # False: it is dropped (load generators that only time)
        self.keep_results = keep_results
        self.n = params.n
        self.max_w, self.max_h = max_width, max_height
        self.max_batch = max(1, int(max_batch))
        self.arena_bytes = int(arena_bytes)
        fixed = max_slots * _Slot.fixed_bytes(self.n, max_width, max_height, self.max_batch)
        if fixed >= self.arena_bytes:
            raise ValueError(f"arena of {self.arena_bytes} bytes cannot hold the slots' fixed buffers ({fixed})")
        self.fixed_bytes = fixed
        # intersections per pixel used to size a launch's bins; raised to the largest ratio any finished
        # launch reported (x 1.1), so overflow re-admissions die out after a few requests
        self.ipp = float(intersections_per_pixel)
        self.slots = [_Slot(self.n, max_width, max_height, self.max_batch, device) for _ in range(max_slots)]
        self.arena = _Arena(self.arena_bytes - fixed, device)
        self.queue: Deque[Request] = collections.deque()
        self.finished: List[Request] = []
        self._next = 0
        self.device = device
        self.launches = 0
        self._pending = []  # (offset, bytes, event): blocks whose result copies are still running

    @property
    def arena_used(self) -> int:
        """Bytes of the budget in use: the slots' fixed buffers plus the admitted blocks."""
        return self.fixed_bytes + self.arena.used

    # ---- client side -------------------------------------------------------------------------
    def submit(self, cam, arrival: Optional[float] = None) -> Request:
        if cam.width > self.max_w or cam.height > self.max_h:
            raise ValueError("resolution above the server's maximum")
        r = Request(self._next, cam, time.perf_counter() if arrival is None else arrival)
        self._next += 1
        self.queue.append(r)
        return r

    # ---- scheduler -----------------------------------------------------------------------------
    def _layout(self, V: int, W: int, H: int, capacity: int):
        """Byte offsets of a launch's block: ids, bin_sort workspace, rgb, depth, normal."""
        tiles = ((W + 15) // 16) * ((H + 15) // 16)
        ws = _lib.lib().cgv2_bin_sort_workspace(capacity, V, tiles, self.n)
        px = V * W * H
        parts = [4 * max(capacity, 1), ws, 12 * px, 4 * px, 12 * px]
        offs, o = [], 0
        for b in parts:
            offs.append(o)
            o += _up(b)
        return offs, parts, o

    def _launch(self, slot: _Slot, reqs: List[Request], off: int, nbytes: int, capacity: int):
        """Binds the launch's block and enqueues project -> bin_sort -> render_fwd (no allocation)."""
        V = len(reqs)
        W, H = reqs[0].cam.width, reqs[0].cam.height
        offs, parts, _ = self._layout(V, W, H, capacity)
        A = self.arena
        ids = A.view(off + offs[0], parts[0], torch.int32, (max(capacity, 1),))
        ws = A.view(off + offs[1], parts[1], torch.uint8, (parts[1],))
        rgb = A.view(off + offs[2], parts[2], torch.float32, (V, 3, H, W))
        depth = A.view(off + offs[3], parts[3], torch.float32, (V, H, W))
        normal = A.view(off + offs[4], parts[4], torch.float32, (V, 3, H, W))
        eng = slot.eng
        L = _Launch()
        L.reqs, L.slot, L.off, L.nbytes, L.capacity, L.W, L.H = list(reqs), slot, off, nbytes, capacity, W, H
        with torch.cuda.stream(slot.stream):
            eng.bind_bins(ids, ws, capacity)
            eng.bind_images(rgb=rgb, depth=depth, normal=normal)
            eng.status.zero_()
            cams = _lib.camera_array([r.cam for r in reqs])
            # an engine for max_batch views runs V <= max_batch views of the call's size
            eng_V = eng.V
            eng.V = V
            try:
                eng.project(self.params, cams)
                eng.bin_sort(cams)
                eng.render(cams)
            finally:
                eng.V = eng_V
            slot.host[0:1].copy_(eng.status, non_blocking=True)
            slot.host[1:2].copy_(eng.needed, non_blocking=True)
            L.event = torch.cuda.Event()
            L.event.record(slot.stream)
        for v, r in enumerate(reqs):
            r._launch, r._view = L, v
            r.result = dict(rgb=rgb[v], depth=depth[v], normal=normal[v])
        slot.launch = L
        self.launches += 1

    def _batch(self) -> List[Request]:
        """The head of the queue and up to max_batch - 1 later requests of its resolution (among the
        next 4 max_batch queued)."""
        head = self.queue[0]
        out = [head]
        if self.max_batch > 1:
            for k, r in enumerate(self.queue):
                if k == 0:
                    continue
                if len(out) == self.max_batch or k >= 4 * self.max_batch:
                    break
                if r.cam.width == head.cam.width and r.cam.height == head.cam.height and r.tries == head.tries:
                    out.append(r)
        return out

    def poll(self) -> int:
        """Retire finished launches, then admit as many queued requests as slots and memory allow.
        Returns the number of requests still queued or running."""
        now = time.perf_counter()
        if self._pending:
            keep = []
            for off, nb, ev in self._pending:
                if ev.query():
                    self.arena.release(off, nb)
                else:
                    keep.append((off, nb, ev))
            self._pending = keep
        for slot in self.slots:
            L = slot.launch
            if L is None or not L.event.query():
                continue
            over = int(slot.host[0]) != 0
            need = int(slot.host[1])
            slot.launch = None
            px = sum(r.cam.width * r.cam.height for r in L.reqs)
            self.ipp = max(self.ipp, 1.1 * need / max(px, 1))
            if over:
                # bins too small: re-admit first, each request sized for the whole launch's need
                self.arena.release(L.off, L.nbytes)
                for r in reversed(L.reqs):
                    r.capacity = int(need * 1.05) + 1024
                    r.result, r._launch = None, None
                    r.tries += 1
                    self.queue.appendleft(r)
                continue
            for r in L.reqs:
                r.done_t = now
                r._launch = None
                self.finished.append(r)
            if self.keep_results:
                # the results leave the arena: copies owned by the requests, made on the slot's stream; the
                # block is given back once the copies have run
                with torch.cuda.stream(slot.stream):
                    for r in L.reqs:
                        r.result = {k: t.clone() for k, t in r.result.items()}
                    ev = torch.cuda.Event()
                    ev.record(slot.stream)
                self._pending.append((L.off, L.nbytes, ev))
            else:
                for r in L.reqs:
                    r.result = None
                self.arena.release(L.off, L.nbytes)
        while self.queue:
            slot = next((s for s in self.slots if s.launch is None), None)
            if slot is None:
                break
            reqs = self._batch()
            for r in reqs:
                if r.tries == 0:
                    r.capacity = int(self.ipp * r.cam.width * r.cam.height) + 4096
            cap = sum(r.capacity for r in reqs) if reqs[0].tries == 0 else max(r.capacity for r in reqs)
            W, H = reqs[0].cam.width, reqs[0].cam.height
            _, _, nbytes = self._layout(len(reqs), W, H, cap)
            if _up(nbytes) > self.arena.size and len(reqs) == 1:
                self.queue.popleft()
                r = reqs[0]
                r.error = "request exceeds the arena"
                r.done_t = now
                self.finished.append(r)
                continue
            off = self.arena.alloc(nbytes)
            if off is None and len(reqs) > 1:
                reqs = reqs[:1]
                cap = reqs[0].capacity
                _, _, nbytes = self._layout(1, W, H, cap)
                off = self.arena.alloc(nbytes)
            if off is None:
                break  # wait for memory (FIFO: no overtaking)
            for r in reqs:
                self.queue.remove(r)
                r.admitted = time.perf_counter()
            self._launch(slot, reqs, off, nbytes, cap)
        return len(self.queue) + sum(s.launch is not None for s in self.slots)

    def drain(self):
        while self.poll() or self._pending:
            time.sleep(50e-6)

    def render_alone(self, cam):
        """One request through an otherwise idle server (reference for the alone-vs-mix check)."""
        r = self.submit(cam)
        self.drain()
        return r


def fixed_bytes(n: int, max_slots: int = 4, max_width: int = 3840, max_height: int = 2160, max_batch: int = 1):
    """Bytes of a server's budget its slots take before any request is admitted."""
    return max_slots * _Slot.fixed_bytes(n, max_width, max_height, max(1, max_batch))


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
