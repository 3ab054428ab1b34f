"""Continuous-batching query server for resident neural fields.

Requests (field id, points[m, n]) arrive from any thread.  A scheduler
thread
  * admits requests in arrival order while the device arena has room for
    their inputs and outputs (memory admission; requests larger than the
    chunk limit are split, so any size fits a bounded arena),
  * copies admitted chunks to the GPU on a copy stream while the previous
    batch computes on the compute stream,
  * launches one fused multi-field query (``spx_field_query_batched``) over
    every uploaded chunk, up to a point budget (the batch mixes fields and
    requests of any size),
  * copies results back, frees their arena ranges, and completes a request
    once all of its chunks are back, stamping its latency.
Requests that arrive while batches are on the GPU join the next batch as
soon as memory frees up.  Every point is computed independently of the
batch it lands in, so a request's result is the same alone and in a mix.

The device side is behind a small backend interface; ``GpuBackend`` drives
the library, and the tests use a CPU backend to exercise admission,
chunking, back-pressure and failure handling without a GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures
import itertools
import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


class RequestError(RuntimeError):
    pass


@dataclass
class Request:
    rid: int
    field: int
    pts: np.ndarray
    t_submit: float
    deadline: Optional[float]
    out: Optional[np.ndarray] = None
    chunks_left: int = 0
    t_done: Optional[float] = None
    error: Optional[str] = None
    _event: threading.Event = field(default_factory=threading.Event, repr=False)

    def wait(self, timeout: Optional[float] = None) -> np.ndarray:
        if not self._event.wait(timeout):
            raise TimeoutError(f"request {self.rid} not done")
        if self.error:
            raise RequestError(self.error)
        return self.out

    @property
    def done(self) -> bool:
        return self._event.is_set()

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_submit


@dataclass
class Chunk:
    req: Request
    lo: int
    hi: int
    off: int = -1       # arena offset of the inputs; outputs follow
    nbytes: int = 0
    up: object = None   # backend handle of the upload
    down: object = None
    copy: object = None  # future of the result copy into the request


class Arena:
    """First-fit allocator of byte ranges in a fixed device buffer."""

    ALIGN = 256

    def __init__(self, capacity: int):
        self.capacity = capacity
        self.free = [(0, capacity)]  # sorted, coalesced (offset, size)

    def alloc(self, nbytes: int) -> Optional[int]:
        n = (nbytes + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                if s == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, s - n)
                return o
        return None

    def release(self, off: int, nbytes: int) -> None:
        n = (nbytes + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    @property
    def free_bytes(self) -> int:
        return sum(s for _, s in self.free)


_DONE = concurrent.futures.Future()
_DONE.set_result(None)


class Server:
    COPY_ASIDE_BYTES = 1 << 20  # results at least this large are copied out on a worker thread

    def __init__(self, backend, field_dims: List[int], field_outs: List[int], arena_bytes: int = 1 << 30,
                 chunk_points: int = 1 << 18, batch_points: int = 1 << 21, max_inflight: int = 2):
        self.backend = backend
        self.dims, self.outs = list(field_dims), list(field_outs)
        self.arena = Arena(arena_bytes)
        backend.alloc_arena(arena_bytes)
        self.chunk_points, self.batch_points, self.max_inflight = chunk_points, batch_points, max_inflight
        # Clients hand chunks over through `incoming` (a deque: appends and
        # pops are atomic) and wake the scheduler; only the scheduler thread
        # touches the other queues, so submitting never waits for it.
        self.incoming: collections.deque = collections.deque()
        self._wake = threading.Event()
        self.pending: collections.deque = collections.deque()   # chunks waiting for memory
        self.uploading: List[Chunk] = []
        self.ready: List[Chunk] = []
        self.inflight: List[tuple] = []                           # (handle, chunks)
        self.downloading: List[Chunk] = []
        self.finishing: List[Chunk] = []                          # results being copied out
        self._copier = concurrent.futures.ThreadPoolExecutor(max_workers=2, thread_name_prefix="spx-results")
        self.completed: List[Request] = []
        self._ids = itertools.count()
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self.batches = 0
        self.batch_sizes: List[int] = []

    # ------------------------------------------------------------- client side

    def submit(self, field_id: int, pts: np.ndarray, timeout: Optional[float] = None) -> Request:
        pts = np.ascontiguousarray(pts, np.float32)
        now = time.perf_counter()
        rid = next(self._ids)
        if not (0 <= field_id < len(self.dims)):
            r = Request(rid, field_id, pts, now, None, error=f"unknown field {field_id}")
            r.t_done = now
            r._event.set()
            return r
        if pts.ndim != 2 or pts.shape[1] != self.dims[field_id]:
            raise ValueError(f"points must be [m, {self.dims[field_id]}]")
        m = pts.shape[0]
        r = Request(rid, field_id, pts, now, None if timeout is None else now + timeout)
        # fault the result's pages in here, on the client's thread: a first
        # touch by the scheduler's copy would run at page-fault speed
        r.out = np.zeros((m, self.outs[field_id]), np.float32)
        r.out.fill(0.0)
        chunks = [Chunk(r, lo, min(lo + self.chunk_points, m)) for lo in range(0, m, self.chunk_points)]
        r.chunks_left = len(chunks)
        if not chunks:
            r.t_done = now
            r._event.set()
            return r
        self.incoming.extend(chunks)
        self._wake.set()
        return r

    # ------------------------------------------------------------- scheduler

    def start(self) -> "Server":
        self._thread = threading.Thread(target=self._loop, name="spx-scheduler", daemon=True)
        self._thread.start()
        return self

    def stop(self) -> None:
        self._stop = True
        self._wake.set()
        if self._thread:
            self._thread.join()
        self._copier.shutdown(wait=True)

    def _fail(self, req: Request, msg: str) -> None:
        if not req.done:
            req.error = msg
            req.t_done = time.perf_counter()
            req._event.set()
            self.completed.append(req)

    def _chunk_bytes(self, c: Chunk) -> int:
        m = c.hi - c.lo
        return (m * self.dims[c.req.field] * 4 + 255) // 256 * 256 + m * self.outs[c.req.field] * 4

    def _admit(self) -> bool:
        progress = False
        now = time.perf_counter()
        while self.pending:
            c = self.pending[0]
            if c.req.done:  # failed earlier
                self.pending.popleft()
                progress = True
                continue
            if c.req.deadline is not None and now > c.req.deadline:
                self.pending.popleft()
                self._fail(c.req, "timed out waiting for memory")
                progress = True
                continue
            nb = self._chunk_bytes(c)
            if nb > self.arena.capacity:
                self.pending.popleft()
                self._fail(c.req, "chunk larger than the arena")
                progress = True
                continue
            off = self.arena.alloc(nb)
            if off is None:
                break  # back-pressure: wait for memory to free up
            self.pending.popleft()
            c.off, c.nbytes = off, nb
            c.up = self.backend.upload(off, c.req.pts[c.lo:c.hi])
            self.uploading.append(c)
            progress = True
        return progress

    def _launch(self) -> bool:
        still = []
        for c in self.uploading:
            try:
                up = self.backend.done(c.up)
            except Exception as e:  # the upload failed: its request fails, the server keeps going
                self.arena.release(c.off, c.nbytes)
                self._fail(c.req, f"upload failed: {e}")
                continue
            (self.ready if up else still).append(c)
        self.uploading = still
        if not self.ready or len(self.inflight) >= self.max_inflight:
            return False
        batch, total = [], 0
        while self.ready and (not batch or total + (self.ready[0].hi - self.ready[0].lo) <= self.batch_points):
            c = self.ready.pop(0)
            batch.append(c)
            total += c.hi - c.lo
        items = []
        for c in batch:
            m = c.hi - c.lo
            in_bytes = (m * self.dims[c.req.field] * 4 + 255) // 256 * 256
            items.append((c.req.field, c.off, c.off + in_bytes, m))
        try:
            h = self.backend.launch(items)
        except Exception as e:  # the batch fails; its requests fail, the server keeps going
            for c in batch:
                self.arena.release(c.off, c.nbytes)
                self._fail(c.req, f"launch failed: {e}")
            return True
        # results come back on their own stream as soon as the batch finishes
        for c, (_, _, out_off, m) in zip(batch, items):
            c.down = self.backend.download(out_off, (m, self.outs[c.req.field]), after=h)
            self.downloading.append(c)
        self.inflight.append((h, batch))
        self.batches += 1
        self.batch_sizes.append(total)
        return True

    def _collect(self) -> bool:
        progress = False
        keep = [(h, b) for h, b in self.inflight if not self.backend.done(h)]
        progress |= len(keep) != len(self.inflight)
        self.inflight = keep
        keep = []
        for c in self.downloading:
            if self.backend.done(c.down):
                if not c.req.done:
                    dst, src = c.req.out[c.lo:c.hi], self.backend.result(c.down)
                    if dst.nbytes >= self.COPY_ASIDE_BYTES:
                        # large results are copied out on a worker; the arena
                        # range is released once the copy has finished
                        c.copy = self._copier.submit(np.copyto, dst, src)
                    else:
                        np.copyto(dst, src)
                        c.copy = _DONE
                    self.finishing.append(c)
                else:
                    self.arena.release(c.off, c.nbytes)
                progress = True
            else:
                keep.append(c)
        self.downloading = keep
        keep = []
        for c in self.finishing:
            if not c.copy.done():
                keep.append(c)
                continue
            self.arena.release(c.off, c.nbytes)
            progress = True
            if c.req.done:
                continue
            err = c.copy.exception()
            if err is not None:
                self._fail(c.req, f"result copy failed: {err}")
                continue
            c.req.chunks_left -= 1
            if c.req.chunks_left == 0:
                c.req.t_done = time.perf_counter()
                c.req._event.set()
                self.completed.append(c.req)
        self.finishing = keep
        return progress

    def _loop(self) -> None:
        while not self._stop:
            self._wake.clear()  # a submit after this point wakes the next wait
            while self.incoming:
                self.pending.append(self.incoming.popleft())
            progress = self._admit()
            progress |= self._launch()
            progress |= self._collect()
            if not progress:
                idle = not (self.pending or self.uploading or self.ready or self.inflight or self.downloading
                            or self.finishing)
                self._wake.wait(timeout=0.01 if idle else 2e-5)


class GpuBackend:
    """Drives libspx on one GPU: an arena in device memory with a pinned host
    mirror, and three streams of default priority: uploads, compute and
    downloads (a download waits for its batch without holding up the next
    uploads)."""

    RING = 4          # segment tables in flight (the server keeps <= 2 batches in flight)
    MAX_SEGS = 4096

    def __init__(self, fields, device="cuda"):
        import torch

        from . import spx
        self.torch, self.spx = torch, spx
        self.device = device
        self.fields = fields  # list of spx.spx_field (host structs)
        blob = spx.as_bytes(fields)
        self.fields_dev = torch.frombuffer(bytearray(blob), dtype=torch.uint8).to(device)
        self.copy = torch.cuda.Stream(device=device)
        self.compute = torch.cuda.Stream(device=device)
        self.back = torch.cuda.Stream(device=device)
        n = 40 * self.MAX_SEGS
        self.seg_pinned = [torch.empty(n, dtype=torch.uint8, pin_memory=True) for _ in range(self.RING)]
        self.seg_dev = [torch.empty(n, dtype=torch.uint8, device=device) for _ in range(self.RING)]
        self.seg_next = 0
        self.pool = concurrent.futures.ThreadPoolExecutor(max_workers=4, thread_name_prefix="spx-upload")

    def alloc_arena(self, nbytes: int) -> None:
        t = self.torch
        self.arena = t.empty(nbytes, dtype=t.uint8, device=self.device)
        self.host_in = t.empty(nbytes, dtype=t.uint8, pin_memory=True)
        self.host_out = t.empty(nbytes, dtype=t.uint8, pin_memory=True)
        self.base = self.arena.data_ptr()

    def _event(self, stream):
        e = self.torch.cuda.Event()
        e.record(stream)
        return e

    def upload(self, off: int, pts: np.ndarray):
        """Stage the points in the pinned mirror and copy them to the arena,
        on a worker thread (the host copy is the scheduler's largest cost)."""
        return self.pool.submit(self._upload, off, pts)

    def _upload(self, off: int, pts: np.ndarray):
        n = pts.nbytes
        dst = self.host_in[off:off + n].numpy()
        dst[:] = pts.view(np.uint8).reshape(-1)
        with self.torch.cuda.stream(self.copy):
            self.arena[off:off + n].copy_(self.host_in[off:off + n], non_blocking=True)
            return self._event(self.copy)

    def launch(self, items):
        t, spx = self.torch, self.spx
        if len(items) > self.MAX_SEGS:
            raise ValueError("too many segments in one batch")
        segs, first = [], 0
        for f, in_off, out_off, m in items:
            s = spx.spx_segment()
            s.pts, s.out = self.base + in_off, self.base + out_off
            s.count, s.first_tile, s.field = m, first, f
            segs.append(s)
            first += (m + 15) // 16
        blob = np.frombuffer(spx.as_bytes(segs), np.uint8)
        k = self.seg_next
        self.seg_next = (k + 1) % self.RING
        self.seg_pinned[k][:blob.size].numpy()[:] = blob
        with t.cuda.stream(self.compute):
            self.compute.wait_stream(self.copy)  # every admitted upload is before this point
            dev = self.seg_dev[k][:blob.size]
            dev.copy_(self.seg_pinned[k][:blob.size], non_blocking=True)
            spx.spx_field_query_batched(self.fields_dev, len(self.fields), dev, len(segs), first, stream=self.compute)
            return self._event(self.compute)

    def download(self, off: int, shape, after):
        n = int(np.prod(shape)) * 4
        with self.torch.cuda.stream(self.back):
            self.back.wait_event(after)
            self.host_out[off:off + n].copy_(self.arena[off:off + n], non_blocking=True)
            ev = self._event(self.back)
        return (ev, off, shape)

    def done(self, h) -> bool:
        if isinstance(h, concurrent.futures.Future):
            if not h.done():
                return False
            h = h.result()  # re-raises a failed upload
        ev = h[0] if isinstance(h, tuple) else h
        return ev.query()

    def result(self, h) -> np.ndarray:
        """A view of the downloaded result in the pinned mirror; valid until
        its arena range is released (the server copies it out first)."""
        _, off, shape = h
        n = int(np.prod(shape)) * 4
        return self.host_out[off:off + n].numpy().view(np.float32).reshape(shape)
