"""Serving: continuous batching of persistence-diagram requests.

Requests (a float32 field each, grids of mixed and anisotropic sizes) arrive
over time. Several workers, each with its own HIP stream and library context,
share one queue. A worker that becomes free takes the waiting requests, in
arrival order, as long as the batch's super grid (the layout of
dms_batch_layout) stays within its vertex budget -- the device memory of a
batch grows with that footprint -- uploads their fields and computes all
their diagrams in one batched run (dms_diagram_batch). While one worker's
batch is on the GPU, requests that arrive are admitted by the next worker
that frees up, so the batches of different workers overlap on the device.
Results stay on the device (the pairs tensors of each request).

Each result is the diagram the request has alone (the batch layout separates
grids by separator planes; see include/dms.h), which the serving test checks.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import dms


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the trace
    host_field: torch.Tensor  # float32 [nz, ny, nx], pinned host memory
    admitted: float = -1.0
    done: float = -1.0
    result: dict | None = None
    batch: int = -1


@dataclass
class ServerConfig:
    workers: int = 2
    budget_vertices: int = 1 << 25   # super-grid vertices per batch
    max_items: int = 512
    cross: tuple = (0, 0)
    z_quantum: int = 16
    use_graph: bool = False


@dataclass
class TraceStats:
    wall_s: float
    latencies_ms: np.ndarray
    # (worker, items, super vertices, real vertices, seconds, start s, end s), times from the trace start
    batches: list = field(default_factory=list)

    @property
    def req_per_s(self) -> float:
        return len(self.latencies_ms) / self.wall_s

    def pct(self, q: float) -> float:
        return float(np.percentile(self.latencies_ms, q))


class Server:
    def __init__(self, cfg: ServerConfig | None = None, device: int = 0):
        self.cfg = cfg or ServerConfig()
        if self.cfg.use_graph and self.cfg.workers > 1:
            # a stream capture fails if another thread allocates or synchronises on
            # the device meanwhile, so graph replay is for a single worker
            raise ValueError("use_graph needs workers == 1")
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.cfg.workers)]
        self.ctxs = [dms.Context(device, stream=s) for s in self.streams]
        self.lock = threading.Condition()
        self.queue: collections.deque[Request] = collections.deque()
        self.closed = False
        self.error: BaseException | None = None

    def close(self):
        for c in self.ctxs:
            c.close()

    def warmup(self, requests: list[Request]):
        """Run the given requests (arrival times ignored) through every
        worker's context once before serving, so that the device buffers a
        batch needs are allocated before the first real request arrives."""
        for w, (ctx, stream) in enumerate(zip(self.ctxs, self.streams)):
            with torch.cuda.stream(stream):
                batch = [Request(r.rid, 0.0, r.host_field) for r in requests]
                self.queue.extend(batch)
                while self.queue:
                    with self.lock:
                        take = self._take_batch()
                    dev = [r.host_field.to(f"cuda:{self.device}", non_blocking=True) for r in take]
                    ctx.diagram_batch(dev, cross=self.cfg.cross, z_quantum=self.cfg.z_quantum,
                                      use_graph=self.cfg.use_graph)
            stream.synchronize()

    # ---- admission ----
    def _take_batch(self) -> list[Request]:
        """Called with the lock held and the queue non-empty: FIFO requests
        while the batch's super grid fits the vertex budget. Boxes are taken
        while their footprint (sides + 1) stays below 3/4 of the budget, then
        the exact layout is checked and the last ones are handed back until
        it fits."""
        budget = self.cfg.budget_vertices
        batch = [self.queue.popleft()]
        foot = _footprint(batch[0])
        while self.queue and len(batch) < self.cfg.max_items:
            f = _footprint(self.queue[0])
            if foot + f > 0.75 * budget:
                break
            foot += f
            batch.append(self.queue.popleft())
        while len(batch) > 1:
            (X, Y, Z), _ = dms.batch_layout([tuple(r.host_field.shape) for r in batch], self.cfg.cross,
                                            self.cfg.z_quantum)
            if X * Y * Z <= budget:
                break
            self.queue.appendleft(batch.pop())
        return batch

    def _worker(self, w: int, t0: float, stats: TraceStats):
        ctx, stream = self.ctxs[w], self.streams[w]
        try:
            with torch.cuda.stream(stream):
                while True:
                    with self.lock:
                        while not self.queue and not self.closed:
                            self.lock.wait()
                        if not self.queue and self.closed:
                            return
                        batch = self._take_batch()
                    now = time.perf_counter() - t0
                    for r in batch:
                        r.admitted = now
                    dev = [r.host_field.to(f"cuda:{self.device}", non_blocking=True) for r in batch]
                    tb = time.perf_counter()
                    out = ctx.diagram_batch(dev, cross=self.cfg.cross, z_quantum=self.cfg.z_quantum,
                                            use_graph=self.cfg.use_graph)
                    done = time.perf_counter()
                    info = ctx.batch_info()
                    with self.lock:
                        stats.batches.append((w, len(batch), info[0] * info[1] * info[2], info[3], done - tb,
                                              tb - t0, done - t0))
                    for r, o in zip(batch, out):
                        r.result = o
                        r.done = done - t0
                        r.batch = len(stats.batches)
        except BaseException as e:  # surfaced by run_trace
            self.error = e
            with self.lock:
                self.closed = True
                self.lock.notify_all()

    def run_trace(self, requests: list[Request]) -> TraceStats:
        """Replay requests at their arrival times; returns when all are done."""
        requests = sorted(requests, key=lambda r: r.arrival)
        stats = TraceStats(0.0, np.zeros(0))
        self.closed = False
        t0 = time.perf_counter()
        threads = [threading.Thread(target=self._worker, args=(w, t0, stats), daemon=True)
                   for w in range(self.cfg.workers)]
        for t in threads:
            t.start()
        for r in requests:
            wait = r.arrival - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            with self.lock:
                if self.closed:
                    break
                self.queue.append(r)
                self.lock.notify()
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        for t in threads:
            t.join()
        if self.error is not None:
            raise self.error
        torch.cuda.synchronize(self.device)
        stats.wall_s = time.perf_counter() - t0
        stats.latencies_ms = np.array([(r.done - r.arrival) * 1e3 for r in requests])
        return stats


def _footprint(r: Request) -> int:
    nz, ny, nx = r.host_field.shape
    return (nx + 1) * (ny + 1) * (nz + 1)


def make_requests(specs, fields) -> list[Request]:
    """specs: [(arrival_s, shape (nz, ny, nx), seed)]; fields: the matching
    numpy arrays (any iterable). All fields live in one pinned host buffer."""
    sizes = [int(np.prod(shape)) for _, shape, _ in specs]
    big = torch.empty(sum(sizes), dtype=torch.float32).pin_memory()
    out, off = [], 0
    for i, ((arr, shape, _seed), f, n) in enumerate(zip(specs, fields, sizes)):
        view = big[off: off + n].view(*shape)
        view.copy_(torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)))
        out.append(Request(i, float(arr), view))
        off += n
    return out


def run_plain(requests: list[Request], device: int = 0) -> float:
    """The plain pipeline on the same requests, one after another on one
    context (no batching, arrivals ignored); returns requests per second."""
    ctx = dms.Context(device)
    try:
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        for r in requests:
            ctx.diagram(r.host_field.to(f"cuda:{device}", non_blocking=True))
        torch.cuda.synchronize(device)
        return len(requests) / (time.perf_counter() - t0)
    finally:
        ctx.close()
