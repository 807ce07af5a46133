"""Serving neighbor-build requests with continuous batching.

Requests (one mesh each, both relations wanted) arrive over time.  The server
keeps S execution slots (HIP streams).  Whenever a slot is free, the requests
that have arrived and are waiting are admitted in arrival order while their
reserved device memory fits the budget (the pair/key buffers dominate), and
go out together as one batched launch on that slot; launches on different
slots overlap on the device.  A request that arrives while others run waits
only for the next free slot and for memory.  Results stay resident on the
device until released; latency = completion - arrival.

The executor is pluggable:

* ``GpuExecutor`` uploads each request into a device arena when it arrives,
  runs each batch through the library's batched entry points
  (``mesh_batch_node_neighbors`` / ``mesh_batch_elem_neighbors``) on its
  slot's stream and detects completion with a HIP event;
* ``FakeExecutor`` (tests) runs on the CPU with a simulated clock and
  duration model, so admission and batching logic are testable without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import heapq
import math
import time
from typing import Callable, List, Optional

import numpy as np

from . import binding as _b


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds on the server clock
    conn: np.ndarray        # int32 [n_elem, npe], local ids
    etype: int
    n_vert: int
    reserve: int = 0        # device bytes reserved while in flight (set by the server)
    admitted: float = math.nan
    completed: float = math.nan
    prep: object = None     # executor state once the upload has started

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


def reserve_bytes(n_elem: int, etype: int, n_vert: int) -> int:
    """Device bytes one request holds while in flight: the workspace of one
    call building both relations, both outputs, and its connectivity (the
    library's own sizing, under the tuned options of a mesh of its size)."""
    from . import autotune
    ws, cap_n, cap_e = _b.query("both", n_elem, etype, n_vert, autotune.options_for("both", etype, n_elem))
    npe = _b.NODES_PER_ELEM[etype]
    return ws + 4 * (cap_n + cap_e) + 8 * (n_vert + 1) + 4 * npe * n_elem


class BudgetError(ValueError):
    pass


@dataclasses.dataclass
class BatchHandle:
    slot: int
    requests: List[Request]
    payload: object = None


class FakeExecutor:
    """CPU stand-in: a batch 'runs' for t0 + elements * per_elem seconds of
    simulated time, computed with the CPU oracle (tests only)."""

    def __init__(self, clock, t0=1e-4, per_elem=1e-8, compute: Optional[Callable] = None):
        self.clock = clock
        self.t0, self.per_elem = t0, per_elem
        self.compute = compute
        self.finish = {}

    def submit(self, batch: BatchHandle):
        n = sum(r.n_elem for r in batch.requests)
        self.finish[id(batch)] = self.clock.now() + self.t0 + n * self.per_elem
        if self.compute is not None:
            batch.payload = [self.compute(r) for r in batch.requests]

    def done(self, batch: BatchHandle) -> bool:
        return self.clock.now() >= self.finish[id(batch)]

    def next_completion(self, batch: BatchHandle) -> float:
        return self.finish[id(batch)]

    def results(self, batch: BatchHandle):
        return batch.payload

    def release(self, batch: BatchHandle):
        self.finish.pop(id(batch), None)


class Arena:
    """First-fit allocator of index ranges in one device connectivity buffer
    (host-side bookkeeping only)."""

    def __init__(self, capacity: int, align: int = 64):
        self.capacity, self.align = int(capacity), align
        self.free = [(0, self.capacity)]  # sorted, disjoint (start, length)
        self.used = {}

    def alloc(self, n: int) -> Optional[int]:
        n = max(int(n), 1)
        n = (n + self.align - 1) // self.align * self.align
        for i, (a, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (a + n, ln - n)
                self.used[a] = n
                return a
        return None

    def release(self, a: int):
        n = self.used.pop(a)
        i = 0
        while i < len(self.free) and self.free[i][0] < a:
            i += 1
        self.free.insert(i, (a, n))
        # merge with the neighbours
        if i + 1 < len(self.free) and a + n == self.free[i + 1][0]:
            self.free[i] = (a, n + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)

    def in_use(self) -> int:
        return sum(self.used.values())


class GpuExecutor:
    """Runs each batch on its slot's stream through the batched C entry points.

    The device connectivity arena has a pinned host twin with the same
    offsets.  When a request arrives (``prepare``) it gets an arena range, and
    a worker thread copies its connectivity into the twin range (numpy, no
    GIL held).  The main thread then uploads finished copies oldest first,
    merging requests that are adjacent in the arena into one copy, on a
    separate upload stream, so uploads overlap the batches already running.
    A batch only writes its segment records (which point into the arena) and
    launches; its slot stream waits for its requests' uploads.  A range is
    free again once its batch has completed.  Each slot keeps its device
    buffers across batches (they only grow)."""

    def __init__(self, n_slots: int, device="cuda:0", copy_threads: int = 8, arena_ids: int = 1 << 28):
        import concurrent.futures

        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(n_slots)]
        self.upload = torch.cuda.Stream(self.device)
        self.slot_state = [None] * n_slots  # each slot's BatchBuild of both relations
        self.arena = Arena(arena_ids)
        self.arena_buf = torch.empty(arena_ids, dtype=torch.int32, device=self.device)
        self.pin = torch.empty(arena_ids, dtype=torch.int32, pin_memory=True)
        self.pin_np = self.pin.numpy()
        self.staging = collections.deque()  # prepared, upload not yet issued, in prepare order
        self.pool = concurrent.futures.ThreadPoolExecutor(max(copy_threads, 1))

    def _copy_in(self, conn: np.ndarray, off: int):
        flat = conn.reshape(-1)
        np.copyto(self.pin_np[off:off + flat.size], flat, casting="unsafe")

    def _flush(self, until: Optional[Request] = None):
        """Upload the staged requests whose host copies are done, oldest first;
        with ``until``, first wait for the copies up to that request."""
        runs, flushed = [], []
        while self.staging:
            r = self.staging[0]
            off, fut, _ = r.prep
            if until is None and not fut.done():
                break
            fut.result()  # waits for `until` and its elders; re-raises a failed copy
            self.staging.popleft()
            end = off + self.arena.used[off]  # the range's padding travels along, harmlessly
            if runs and runs[-1][1] == off:
                runs[-1][1] = end
            else:
                runs.append([off, end])
            flushed.append(r)
            if r is until:
                until = None
        if not flushed:
            return
        torch = self.torch
        with torch.cuda.stream(self.upload):
            for a, b in runs:
                self.arena_buf[a:b].copy_(self.pin[a:b], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.upload)
        for r in flushed:
            r.prep[2] = ev

    def prepare(self, r: Request) -> bool:
        """Start staging and uploading r; False if the arena is full now."""
        if r.conn.size > self.arena.capacity:
            raise BudgetError(f"request {r.rid} has {r.conn.size} ids, the arena holds {self.arena.capacity}")
        off = self.arena.alloc(r.conn.size)
        if off is None:
            return False
        r.prep = [off, self.pool.submit(self._copy_in, r.conn, off), None]  # range, host copy, upload event
        self.staging.append(r)
        self._flush()
        return True

    def submit(self, batch: BatchHandle):
        torch = self.torch
        st = self.slot_state[batch.slot]
        s = self.streams[batch.slot]
        desc = [(r.n_elem, r.etype, r.n_vert) for r in batch.requests]
        offs = []
        for r in batch.requests:
            if r.prep[2] is None:
                self._flush(until=r)
            s.wait_event(r.prep[2])
            offs.append(r.prep[0])
        with torch.cuda.stream(s):
            if st is None:
                st = self.slot_state[batch.slot] = _b.BatchBuild("both", desc, self.device, conn_offs=offs,
                                                                 options="tuned")
            else:
                st.reset(desc, s, conn_offs=offs)
            st.launch(self.arena_buf, s)
            ev = torch.cuda.Event()
            ev.record(s)
        batch.payload = {"build": st, "event": ev}

    def done(self, batch: BatchHandle) -> bool:
        return batch.payload["event"].query()

    def next_completion(self, batch: BatchHandle) -> float:
        return math.nan

    def results(self, batch: BatchHandle):
        """Per request: ((node row_ptr, cols), (elem row_ptr, cols)) as host arrays."""
        p = batch.payload
        s = self.streams[batch.slot]
        out = []
        (node_rp, node_cols), (elem_rp, elem_cols) = p["build"].result(s)
        nrp, ncol = node_rp.cpu().numpy(), node_cols.cpu().numpy()
        erp, ecol = elem_rp.cpu().numpy(), elem_cols.cpu().numpy()
        for seg in p["build"].seg_host:
            v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
            a, b = int(nrp[v0]), int(nrp[v0 + nv])
            c, d = int(erp[v0]), int(erp[v0 + nv])
            out.append(((nrp[v0:v0 + nv + 1] - a, ncol[a:b]), (erp[v0:v0 + nv + 1] - c, ecol[c:d])))
        return out

    def check(self, batch: BatchHandle):
        batch.payload["build"].check(self.streams[batch.slot])

    def release(self, batch: BatchHandle):
        # the batch has completed, so the arena ranges it read are free again
        for r in batch.requests:
            if getattr(r, "prep", None) is not None:
                self.arena.release(r.prep[0])
                r.prep = None
        batch.payload = None


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float):
        while self.now() < t:
            pass


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def wait_until(self, t: float):
        self.t = max(self.t, t)


class Server:
    """Continuous batching over ``n_slots`` slots under ``budget_bytes``."""

    def __init__(self, executor, clock, n_slots=4, budget_bytes=64 << 30, max_batch=64,
                 on_complete: Optional[Callable] = None, reserve: Callable = reserve_bytes, max_staged=64):
        self.ex = executor
        self.clock = clock
        self.n_slots = n_slots
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.on_complete = on_complete
        self.reserve = reserve
        self.max_staged = max_staged  # uploads started ahead of admission, at most
        self.admitted = 0
        self.in_use = 0
        self.peak_in_use = 0
        self.batches = 0
        self.batch_sizes = []
        self.waiting = collections.deque()
        self.running = {}  # slot -> BatchHandle

    def _admit_into(self, slot: int) -> Optional[BatchHandle]:
        now = self.clock.now()
        take = []
        staged = hasattr(self.ex, "prepare")
        while self.waiting and self.waiting[0].arrival <= now and len(take) < self.max_batch:
            r = self.waiting[0]
            if self.in_use + r.reserve > self.budget:
                break  # FIFO: the head waits for memory, later ones wait behind it
            if staged and r.prep is None:
                break  # its upload has not started (connectivity arena full)
            self.waiting.popleft()
            self.in_use += r.reserve
            r.admitted = now
            self.admitted += 1
            take.append(r)
        if not take:
            return None
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        b = BatchHandle(slot, take)
        self.ex.submit(b)
        self.running[slot] = b
        self.batches += 1
        self.batch_sizes.append(len(take))
        return b

    def _retire(self, slot: int):
        b = self.running.pop(slot)
        now = self.clock.now()
        for r in b.requests:
            r.completed = now
        if self.on_complete is not None:
            self.on_complete(b, self.ex)
        for r in b.requests:
            self.in_use -= r.reserve
        self.ex.release(b)

    def run(self, requests: List[Request]) -> List[Request]:
        """Serve the requests (sorted by arrival) to completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.reserve = self.reserve(r.n_elem, r.etype, r.n_vert)
            if r.reserve > self.budget:
                raise BudgetError(f"request {r.rid} needs {r.reserve} bytes, budget is {self.budget}")
        self.waiting.extend(reqs)
        prepare = getattr(self.ex, "prepare", None)
        next_prep = 0  # requests are prepared in arrival order as they arrive
        first = self.admitted
        while self.waiting or self.running:
            progressed = False
            if prepare is not None:
                now = self.clock.now()
                while (next_prep < len(reqs) and reqs[next_prep].arrival <= now
                       and next_prep - (self.admitted - first) < self.max_staged):
                    if not prepare(reqs[next_prep]):
                        break  # arena full: retry once a batch has released its ranges
                    next_prep += 1
            for slot in list(self.running):
                if self.ex.done(self.running[slot]):
                    self._retire(slot)
                    progressed = True
            for slot in range(self.n_slots):
                if slot not in self.running and self._admit_into(slot) is not None:
                    progressed = True
            if progressed:
                continue
            # nothing to do right now: advance to the next event
            nxt = [self.ex.next_completion(b) for b in self.running.values()]
            nxt = [t for t in nxt if not math.isnan(t)]
            if self.waiting and self.waiting[0].arrival > self.clock.now():
                nxt.append(self.waiting[0].arrival)
            if nxt:
                self.clock.wait_until(min(nxt))
        return reqs


def latency_summary(reqs: List[Request]):
    lat = np.array([r.latency for r in reqs])
    elems = sum(r.n_elem for r in reqs)
    span = max(r.completed for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "elements": int(elems), "span_s": float(span), "elements_per_s": float(elems / span)}
