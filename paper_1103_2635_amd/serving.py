"""Continuous-batching search server over a resident index.

Requests (a block of queries and a k) arrive over time.  The scheduler keeps
a FIFO of arrived requests and, whenever an execution slot (a HIP stream) is
free and the workspace budget allows it, launches a batch:

  * requests with the same k are coalesced, oldest first, up to
    ``max_batch`` queries;
  * a request larger than ``max_batch`` is split into chunks, each a batch of
    its own (the request completes with its last chunk);
  * a batch is admitted only if its search workspace fits in the memory not
    held by batches in flight (admission by workspace memory);
  * batches on different slots run concurrently on the device.

A request's latency runs from its scheduled arrival to the moment the
scheduler sees its last batch complete, so queueing counts.  The scheduler is
independent of the device: ``GpuExecutor`` runs batches with
``rbc_search`` / ``bf_search`` on torch streams; tests drive it with a fake
executor on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional


@dataclasses.dataclass
class Request:
    rid: int
    offset: int          # first query of the request in the query pool
    m: int               # number of queries
    k: int
    arrival: float       # scheduled arrival time (seconds, trace clock)
    done_at: Optional[float] = None
    chunks_left: int = 0
    results: list = dataclasses.field(default_factory=list)  # (start, idx, dist) per chunk


@dataclasses.dataclass
class Batch:
    k: int
    parts: list          # (request, start within request, count)
    m: int
    ws_bytes: int
    handle: object = None
    slot: int = -1


class Scheduler:
    """Admission, batching and completion bookkeeping (device independent)."""

    def __init__(self, executor, n_slots: int, mem_budget: int, max_batch: int):
        if n_slots < 1 or max_batch < 1:
            raise ValueError("need at least one slot and a positive batch size")
        self.ex = executor
        self.n_slots = n_slots
        self.mem_budget = mem_budget
        self.max_batch = max_batch
        self.pending = collections.deque()   # (request, start, count) not yet launched
        self.free_slots = list(range(n_slots))
        self.in_flight: List[Batch] = []
        self.mem_used = 0
        self.completed: List[Request] = []
        self.max_mem_used = 0
        self.batches_launched = 0
        self.max_concurrent = 0

    def submit(self, req: Request):
        """Queue an arrived request (split into chunks of at most max_batch)."""
        nchunks = (req.m + self.max_batch - 1) // self.max_batch
        req.chunks_left = nchunks
        for c in range(nchunks):
            s = c * self.max_batch
            self.pending.append((req, s, min(self.max_batch, req.m - s)))

    def _form_batch(self):
        """Oldest pending chunk, plus later chunks with the same k while they fit."""
        req, s, cnt = self.pending[0]
        parts = [(req, s, cnt)]
        total = cnt
        rest = collections.deque()
        self.pending.popleft()
        while self.pending:
            r2, s2, c2 = self.pending[0]
            if r2.k == req.k and total + c2 <= self.max_batch:
                parts.append(self.pending.popleft())
                total += c2
            else:
                # keep FIFO order for what is skipped
                rest.append(self.pending.popleft())
        while rest:
            self.pending.appendleft(rest.pop())
        return Batch(k=req.k, parts=parts, m=total, ws_bytes=self.ex.workspace_bytes(total, req.k))

    def launch_ready(self, now: float):
        while self.pending and self.free_slots:
            b = self._form_batch()
            if self.mem_used + b.ws_bytes > self.mem_budget and self.in_flight:
                # does not fit beside the batches in flight: put it back, wait
                for part in reversed(b.parts):
                    self.pending.appendleft(part)
                return
            b.slot = self.free_slots.pop()
            self.mem_used += b.ws_bytes
            self.max_mem_used = max(self.max_mem_used, self.mem_used)
            b.handle = self.ex.launch(b)
            self.in_flight.append(b)
            self.batches_launched += 1
            self.max_concurrent = max(self.max_concurrent, len(self.in_flight))

    def reap(self, now_fn: Callable[[], float]):
        """Retire completed batches; returns the number retired."""
        n = 0
        still = []
        for b in self.in_flight:
            if self.ex.done(b.handle):
                t = now_fn()
                res = self.ex.results(b)
                off = 0
                for (req, s, cnt) in b.parts:
                    req.results.append((s, res[0][off:off + cnt], res[1][off:off + cnt]))
                    off += cnt
                    req.chunks_left -= 1
                    if req.chunks_left == 0:
                        req.done_at = t
                        self.completed.append(req)
                self.ex.release(b)
                self.mem_used -= b.ws_bytes
                self.free_slots.append(b.slot)
                n += 1
            else:
                still.append(b)
        self.in_flight = still
        return n

    def idle(self):
        return not self.pending and not self.in_flight


def replay(sched: Scheduler, requests: List[Request], clock: Callable[[], float],
           sleep: Callable[[float], None] = lambda s: None, poll: float = 20e-6):
    """Open-loop replay: each request is submitted at its scheduled arrival;
    the loop launches and reaps until every request has completed.  Returns
    the requests in completion order."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    i = 0
    t0 = clock()
    while i < len(reqs) or not sched.idle():
        now = clock() - t0
        while i < len(reqs) and reqs[i].arrival <= now:
            sched.submit(reqs[i])
            i += 1
        sched.launch_ready(now)
        sched.reap(lambda: clock() - t0)
        if i < len(reqs) and sched.idle():
            sleep(max(0.0, min(reqs[i].arrival - (clock() - t0), poll)))
        elif not sched.idle():
            sleep(poll)
    return sched.completed


def latency_stats(reqs: List[Request]):
    import numpy as np

    lat = np.array([r.done_at - r.arrival for r in reqs])
    nq = sum(r.m for r in reqs)
    span = max(r.done_at for r in reqs) - min(r.arrival for r in reqs)
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "qps": nq / span if span > 0 else float("inf"),
            "requests": len(reqs), "queries": nq}


class GpuExecutor:
    """Runs batches on torch streams with the library's search entry points.

    ``search(Q, k, out, workspace)`` is called with the slot's stream current.
    Each slot owns, from construction on, a device arena sized for the largest
    batch (``max_batch`` queries, any k <= ``max_k``): the search workspace,
    a block the queries of a multi-request batch are gathered into, the
    outputs, and pinned host buffers the outputs are copied back into on the
    slot's stream.  Serving therefore calls no device allocator, and a batch
    completes when its results are in host memory (the copy counts in the
    latency).  ``results`` returns host tensors."""

    class _Slot:
        pass

    def __init__(self, pool, search_fn, ws_fn, n_slots: int, max_batch: int, max_k: int):
        import torch

        self.torch = torch
        self.pool = pool
        self.search_fn = search_fn
        self.ws_fn = ws_fn
        self.max_batch, self.max_k = max_batch, max_k
        ws_max = max(int(ws_fn(max_batch, k)) for k in range(1, max_k + 1))
        dev = pool.device
        self.slots = []
        for _ in range(n_slots):
            sl = self._Slot()
            sl.stream = torch.cuda.Stream()
            sl.ws = torch.empty(max(1, ws_max), dtype=torch.uint8, device=dev)
            sl.q = torch.empty((max_batch, pool.shape[1]), dtype=pool.dtype, device=dev)
            sl.oi = torch.empty(max_batch * max_k, dtype=torch.int64, device=dev)
            sl.od = torch.empty(max_batch * max_k, dtype=torch.float32, device=dev)
            sl.hi = torch.empty(max_batch * max_k, dtype=torch.int64, pin_memory=True)
            sl.hd = torch.empty(max_batch * max_k, dtype=torch.float32, pin_memory=True)
            sl.ev = torch.cuda.Event()
            self.slots.append(sl)
        torch.cuda.synchronize()

    def workspace_bytes(self, m, k):
        return int(self.ws_fn(m, k))

    def launch(self, b: Batch):
        torch = self.torch
        if b.m > self.max_batch or b.k > self.max_k:
            raise ValueError("batch of %d queries, k=%d exceeds the slot arena (%d, %d)"
                             % (b.m, b.k, self.max_batch, self.max_k))
        sl = self.slots[b.slot]
        sl.stream.wait_stream(torch.cuda.current_stream())
        mk = b.m * b.k
        with torch.cuda.stream(sl.stream):
            if len(b.parts) == 1:
                req, s, cnt = b.parts[0]
                Q = self.pool[req.offset + s:req.offset + s + cnt]
            else:
                Q = sl.q[:b.m]
                torch.cat([self.pool[r.offset + s:r.offset + s + c] for (r, s, c) in b.parts], out=Q)
            out = (sl.oi[:mk].view(b.m, b.k), sl.od[:mk].view(b.m, b.k))
            self.search_fn(Q, b.k, out, sl.ws)
            sl.hi[:mk].copy_(sl.oi[:mk], non_blocking=True)
            sl.hd[:mk].copy_(sl.od[:mk], non_blocking=True)
            sl.ev.record(sl.stream)
        return sl.ev

    def done(self, ev):
        return ev.query()

    def results(self, b: Batch):
        sl = self.slots[b.slot]
        mk = b.m * b.k
        return (sl.hi[:mk].view(b.m, b.k).clone(), sl.hd[:mk].view(b.m, b.k).clone())

    def release(self, b: Batch):
        pass
