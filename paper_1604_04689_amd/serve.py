"""Serving neighbor-build requests with continuous batching.

Requests (one mesh each, both relations wanted) arrive over time.  The server
keeps S execution slots (HIP streams).  Whenever a slot is free, the requests
that have arrived and are waiting are admitted in arrival order while their
reserved device memory fits the budget (the pair/key buffers dominate), and
go out together as one batched launch on that slot; launches on different
slots overlap on the device.  A request that arrives while others run waits
only for the next free slot and for memory; latency = completion - arrival.

Results stay resident on the device: when its batch completes, every request
gets a ``ResultHandle`` (``request.result``) over its slices of the batch's
output tensors, which no later batch overwrites.  The budget keeps counting a
result's bytes until the client calls ``release()`` on it, so results the
client holds on to make later requests wait for memory.  With
``keep_results=False`` (the default) the server releases each result right
after the completion callback has seen it.

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
import contextlib
import dataclasses
import functools
import gc
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
    conn: np.ndarray        # int32 [n_elem, npe], local ids (host array, or a torch device tensor)
    etype: int
    n_vert: int
    reserve: int = 0        # device bytes reserved while in flight (set by the server)
    resident: int = 0       # of which held after completion until the result is released
    admitted: float = math.nan
    completed: float = math.nan
    prep: object = None     # executor state once the upload has started
    result: object = None   # ResultHandle once completed

    @property
    def n_elem(self) -> int:
        return int(self.conn.shape[0])  # numpy array, or a device tensor of the same shape

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


@functools.lru_cache(maxsize=1 << 16)
def output_bytes(n_elem: int, etype: int, n_vert: int) -> int:
    """Device bytes of one request's results (both CSRs at their worst-case
    capacity), held from its launch until the client releases them."""
    npe, k = _b.NODES_PER_ELEM[etype], _b.EDGES_PER_ELEM[etype]
    return 4 * (2 * k * n_elem + npe * n_elem) + 8 * (n_vert + 1)


@functools.lru_cache(maxsize=1 << 16)
def reserve_bytes(n_elem: int, etype: int, n_vert: int) -> int:
    """Device bytes one request holds while in flight: the workspace of one
    call building both relations, both outputs, and its connectivity (the
    library's own sizing, under the tuned options of a mesh of its size).
    The outputs (output_bytes) stay held after completion until released."""
    from . import autotune
    ws, _, _ = _b.query("both", n_elem, etype, n_vert, autotune.options_for("both", etype, n_elem))
    npe = _b.NODES_PER_ELEM[etype]
    return ws + output_bytes(n_elem, etype, n_vert) + 4 * npe * n_elem


class BudgetError(ValueError):
    pass


class ResultHandle:
    """One served request's node and element CSRs, resident where the
    executor left them (device tensors for the GPU executor) until
    ``release()``.  ``node()`` / ``elem()`` give (row_ptr, cols) views of
    the batch's output (row_ptr still holding the batch's offsets; subtract
    ``node_base`` / ``elem_base``, or use ``node_csr()`` / ``elem_csr()``
    which do); ``to_host()`` copies both CSRs, rebased, to numpy arrays."""

    def __init__(self, node, elem, node_base, elem_base, on_release):
        # node / elem: (row_ptr, cols), or a callable that makes them on first
        # use (the GPU executor's views cost microseconds per request, which a
        # client that only releases never pays)
        self._node, self._elem = node, elem
        self.node_base, self.elem_base = node_base, elem_base
        self._on_release = on_release
        self._released = False

    @property
    def released(self) -> bool:
        return self._released

    def _live(self):
        if self._released:
            raise ValueError("result was released")

    def node(self):
        self._live()
        if callable(self._node):
            self._node = self._node()
        return self._node

    def elem(self):
        self._live()
        if callable(self._elem):
            self._elem = self._elem()
        return self._elem

    def node_csr(self):
        rp, cols = self.node()
        return rp - self.node_base, cols

    def elem_csr(self):
        rp, cols = self.elem()
        return rp - self.elem_base, cols

    def to_host(self):
        """((node row_ptr, cols), (elem row_ptr, cols)) as numpy arrays."""
        def host(x):
            return x.cpu().numpy() if hasattr(x, "cpu") else np.asarray(x)
        (nr, nc), (er, ec) = self.node_csr(), self.elem_csr()
        return (host(nr), host(nc)), (host(er), host(ec))

    def release(self):
        """Give the result's memory back (idempotent)."""
        if self._released:
            return
        self._released = True
        self._node = self._elem = None
        cb, self._on_release = self._on_release, None
        if cb is not None:
            cb()


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

    def handles(self, batch: BatchHandle, on_release):
        """One ResultHandle per request over the computed host arrays (None
        entries when there is no compute function)."""
        out = []
        for i, r in enumerate(batch.requests):
            res = batch.payload[i] if batch.payload is not None else ((None, None), (None, None))
            out.append(ResultHandle(res[0], res[1], 0, 0, (lambda r=r: on_release(r))))
        return out

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


def _n_ids(conn) -> int:
    return int(conn.numel()) if hasattr(conn, "numel") else int(conn.size)


def _on_device(conn) -> bool:
    return hasattr(conn, "is_cuda") and conn.is_cuda


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
    free again once its batch has completed.  Each slot keeps its workspace
    across batches (it only grows); a batch's outputs come from a pool of
    output sets and go back to it when every result of the batch has been
    released, so steady serving allocates nothing."""

    COPY_TASK_IDS = 1 << 20  # ids one host-copy task copies at least (fewer, larger tasks)

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
        self._pad = torch.zeros(self.arena.align, dtype=torch.int32, device=self.device)  # fills alignment gaps
        self.pin = torch.empty(arena_ids, dtype=torch.int32, pin_memory=True)
        self.pin_np = self.pin.numpy()
        self.staging = collections.deque()  # prepared, upload not yet issued, in prepare order
        self.pool = concurrent.futures.ThreadPoolExecutor(max(copy_threads, 1))
        self.free_outs = []  # output sets whose results were all released
        self.dev_pending, self.host_pending = [], []  # prepared, upload not started

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
        """Give r an arena range and queue its upload (started by commit());
        False if the arena is full now.  A request whose connectivity is
        already a device tensor is copied into the arena on the upload stream
        (no host staging)."""
        n = _n_ids(r.conn)
        if n > self.arena.capacity:
            raise BudgetError(f"request {r.rid} has {n} ids, the arena holds {self.arena.capacity}")
        off = self.arena.alloc(n)
        if off is None:
            return False
        r.prep = [off, None, None]  # range, host copy, upload event
        (self.dev_pending if _on_device(r.conn) else self.host_pending).append(r)
        return True

    def commit(self):
        """Start the uploads of every request prepared since the last commit:
        device inputs as copies on the upload stream behind one event, host
        inputs as a few worker tasks (each copying several requests into the
        pinned twin), uploaded as their copies finish."""
        torch = self.torch
        if self.dev_pending:
            self.upload.wait_stream(torch.cuda.current_stream(self.device))  # the tensors' producers
            with torch.cuda.stream(self.upload):
                # requests whose arena ranges follow each other go in one
                # concatenation (one launch instead of one copy each); the
                # alignment padding between ranges is filled from a zero
                # buffer and never read
                run, end = [], None
                for r in self.dev_pending + [None]:
                    if r is not None and r.prep[0] == end:
                        run.append(r)
                        end += self.arena.used[r.prep[0]]
                        continue
                    if len(run) > 1 and all(x.conn.dtype == torch.int32 for x in run):
                        parts = []
                        for x in run:
                            parts.append(x.conn.reshape(-1))
                            pad = self.arena.used[x.prep[0]] - _n_ids(x.conn)
                            if pad:
                                parts.append(self._pad[:pad])
                        torch.cat(parts, out=self.arena_buf[run[0].prep[0]:end])
                    else:
                        for x in run:
                            off = x.prep[0]
                            self.arena_buf[off:off + _n_ids(x.conn)].copy_(x.conn.reshape(-1), non_blocking=True)
                    if r is not None:
                        run, end = [r], r.prep[0] + self.arena.used[r.prep[0]]
                ev = torch.cuda.Event()
                ev.record(self.upload)
            for r in self.dev_pending:
                r.prep[2] = ev
            self.dev_pending = []
        if self.host_pending:
            group, ids = [], 0
            for i, r in enumerate(self.host_pending):
                group.append(r)
                ids += r.conn.size
                if ids >= self.COPY_TASK_IDS or i + 1 == len(self.host_pending):
                    fut = self.pool.submit(self._copy_group, [(x.conn, x.prep[0]) for x in group])
                    for x in group:
                        x.prep[1] = fut
                        self.staging.append(x)
                    group, ids = [], 0
            self.host_pending = []
            self._flush()

    def _copy_group(self, items):
        for conn, off in items:
            self._copy_in(conn, off)

    def submit(self, batch: BatchHandle):
        torch = self.torch
        st = self.slot_state[batch.slot]
        s = self.streams[batch.slot]
        desc = [(r.n_elem, r.etype, r.n_vert) for r in batch.requests]
        offs = []
        self.commit()
        waited = set()
        for r in batch.requests:
            if r.prep[2] is None:
                self._flush(until=r)
            if id(r.prep[2]) not in waited:  # requests uploaded together share one event
                waited.add(id(r.prep[2]))
                s.wait_event(r.prep[2])
            offs.append(r.prep[0])
        with torch.cuda.stream(s):
            if st is None:
                st = self.slot_state[batch.slot] = _b.BatchBuild("both", desc, self.device, conn_offs=offs,
                                                                 options="tuned")
            else:
                st.reset(desc, s, conn_offs=offs, outputs=False)
            oset = self._take_outputs(st.output_sizes())
            outs = st.set_outputs(oset["bufs"])  # this batch's results outlive the slot's next batch
            st.launch(self.arena_buf, s)
            ev = torch.cuda.Event()
            ev.record(s)
        oset["refs"] = len(batch.requests)
        batch.payload = {"build": st, "event": ev, "outs": outs, "seg": st.seg_host, "oset": oset}

    def warm(self, requests: List[Request], max_batch: int):
        """Size every slot for the largest batch these requests can form (the
        max_batch largest by directed pairs), and give each slot an output
        set of that size, so that no device allocation happens while
        serving.  Call before the server's clock starts."""
        torch = self.torch
        if not requests:
            return
        big = sorted(requests, key=lambda r: -_b.EDGES_PER_ELEM[r.etype] * r.n_elem)[:max_batch]
        desc = [(r.n_elem, r.etype, r.n_vert) for r in big]
        for i, s in enumerate(self.streams):
            with torch.cuda.stream(s):
                if self.slot_state[i] is None:
                    self.slot_state[i] = _b.BatchBuild("both", desc, self.device, options="tuned")
                else:
                    self.slot_state[i].reset(desc, s, outputs=False)
            self.free_outs.append(self._take_outputs(self.slot_state[i].output_sizes()))
        # the first use of a torch kernel loads its code (up to about 0.1 s,
        # measured inside the serving loop on MI355X): run the row gathers of
        # every batch size once now (torch picks different kernels for few
        # and for many indices)
        nrp, erp = self.free_outs[0]["bufs"][0], self.free_outs[0]["bufs"][2]
        for n in range(1, max_batch + 2):
            self._gather_rows(nrp, erp, np.zeros(n, dtype=np.int64))
        torch.cuda.synchronize(self.device)

    def _take_outputs(self, sizes):
        """An output set (node row_ptr, cols, elem row_ptr, cols) holding at
        least `sizes` entries: a released one when one is large enough, else a
        new one with some headroom.  A set returns to the pool once every
        result handle of its batch is released."""
        for i, o in enumerate(self.free_outs):
            if all(b.numel() >= n for b, n in zip(o["bufs"], sizes)):
                return self.free_outs.pop(i)
        torch = self.torch
        bufs = [torch.empty(int(n * 1.25) + 64, dtype=torch.int32, device=self.device) for n in sizes]
        return {"bufs": bufs, "refs": 0}

    def _put_outputs(self, oset):
        oset["refs"] -= 1
        if oset["refs"] == 0:
            self.free_outs.append(oset)

    def done(self, batch: BatchHandle) -> bool:
        return batch.payload["event"].query()

    def next_completion(self, batch: BatchHandle) -> float:
        return math.nan

    def _bounds(self, batch: BatchHandle):
        """Row starts of every request's slices (one device-to-host copy of
        2 x (requests + 1) entries of the completed batch's row pointers)."""
        p = batch.payload
        if "bounds" not in p:
            p["bounds"] = self._gather_rows(p["outs"][0], p["outs"][2],
                                            np.append(p["seg"]["vert_off"], p["build"].totals["vert"]))
        return p["bounds"]

    def _gather_rows(self, nrp, erp, rows):
        """nrp[rows] and erp[rows] as one (2, len(rows)) host array."""
        torch = self.torch
        idx = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=self.device)
        return torch.stack([nrp.index_select(0, idx), erp.index_select(0, idx)]).cpu().numpy()

    def handles(self, batch: BatchHandle, on_release):
        """One ResultHandle per request: device views into the batch's own
        output tensors, which stay allocated while any handle holds them."""
        p = batch.payload
        b = self._bounds(batch)
        nrp, ncol, erp, ecol = p["outs"]
        out = []
        for i, seg in enumerate(p["seg"]):
            v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
            a, bb, c, d = int(b[0, i]), int(b[0, i + 1]), int(b[1, i]), int(b[1, i + 1])
            r = batch.requests[i]

            def done(r=r, oset=p["oset"]):
                on_release(r)
                self._put_outputs(oset)
            out.append(ResultHandle(lambda v0=v0, nv=nv, a=a, bb=bb: (nrp[v0:v0 + nv + 1], ncol[a:bb]),
                                    lambda v0=v0, nv=nv, c=c, d=d: (erp[v0:v0 + nv + 1], ecol[c:d]), a, c, done))
        return out

    def results(self, batch: BatchHandle):
        """Per request: ((node row_ptr, cols), (elem row_ptr, cols)) as host arrays."""
        p = batch.payload
        nrp, ncol, erp, ecol = (x.cpu().numpy() for x in p["outs"])
        b = self._bounds(batch)
        out = []
        for i, seg in enumerate(p["seg"]):
            v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
            a, bb, c, d = int(b[0, i]), int(b[0, i + 1]), int(b[1, i]), int(b[1, i + 1])
            out.append(((nrp[v0:v0 + nv + 1] - a, ncol[a:bb]), (erp[v0:v0 + nv + 1] - c, ecol[c:d])))
        return out

    def check(self, batch: BatchHandle):
        batch.payload["build"].check(self.streams[batch.slot])

    def release(self, batch: BatchHandle):
        # the batch has completed, so the arena ranges it read are free again;
        # its outputs live on in the result handles that still reference them
        for r in batch.requests:
            if getattr(r, "prep", None) is not None:
                self.arena.release(r.prep[0])
                r.prep = None
        batch.payload = None


@contextlib.contextmanager
def frozen_gc():
    """Collect once, then keep every object alive now out of the cyclic
    collector's passes until the block ends.  A full pass over all the
    objects a serving process holds (meshes, tensors, requests) takes tens of
    milliseconds and, inside the serving loop, shows as a latency outlier;
    enter this before the clock starts."""
    gc.collect()
    gc.freeze()
    try:
        yield
    finally:
        gc.unfreeze()


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
                 on_complete: Optional[Callable] = None, reserve: Callable = reserve_bytes, max_staged=None,
                 keep_results: bool = False, resident: Callable = output_bytes):
        self.ex = executor
        self.clock = clock
        self.n_slots = n_slots
        self.budget = budget_bytes
        self.max_batch = max_batch
        self.on_complete = on_complete
        self.reserve = reserve
        # uploads started ahead of admission, at most (default: enough to fill every slot twice)
        self.max_staged = max_staged if max_staged is not None else 2 * n_slots * max_batch
        self.keep_results = keep_results
        self.resident_fn = resident
        self.admitted = 0
        self.in_use = 0           # reserved bytes: in-flight requests and unreleased results
        self.resident_bytes = 0   # of which held by completed, unreleased results
        self.unreleased = 0
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

    def _release_result(self, r: Request):
        self.in_use -= r.resident
        self.resident_bytes -= r.resident
        self.unreleased -= 1

    def _retire(self, slot: int):
        b = self.running.pop(slot)
        now = self.clock.now()
        for r in b.requests:
            r.completed = now
            self.in_use -= r.reserve - r.resident  # the workspace and inputs are free; results stay
            self.resident_bytes += r.resident
            self.unreleased += 1
        for r, h in zip(b.requests, self.ex.handles(b, self._release_result)):
            r.result = h
        if self.on_complete is not None:
            self.on_complete(b, self.ex)
        self.ex.release(b)
        if not self.keep_results:
            for r in b.requests:
                r.result.release()

    def run(self, requests: List[Request]) -> List[Request]:
        """Serve the requests (sorted by arrival) to completion."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.reserve = self.reserve(r.n_elem, r.etype, r.n_vert)
            r.resident = min(self.resident_fn(r.n_elem, r.etype, r.n_vert), r.reserve)
            if r.reserve > self.budget:
                raise BudgetError(f"request {r.rid} needs {r.reserve} bytes, budget is {self.budget}")
        self.waiting.extend(reqs)
        prepare = getattr(self.ex, "prepare", None)
        commit = getattr(self.ex, "commit", None)
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
                if commit is not None:
                    commit()
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
            elif not self.running and self.waiting and self.in_use + self.waiting[0].reserve > self.budget:
                # nothing runs, and unreleased results hold the memory the next request needs
                raise BudgetError(f"request {self.waiting[0].rid} waits for {self.waiting[0].reserve} bytes, but "
                                  f"{self.resident_bytes} bytes of the {self.budget}-byte budget are held by "
                                  f"{self.unreleased} unreleased results")
        return reqs


def latency_summary(reqs: List[Request]):
    lat = np.array([r.latency for r in reqs])
    arr = np.array([r.arrival for r in reqs])
    elems = sum(r.n_elem for r in reqs)
    span = max(r.completed for r in reqs) - arr.min()
    p99 = float(np.percentile(lat, 99))
    tail = arr[lat >= p99] - arr.min()  # when the slowest 1% arrived (a stall shows as a narrow window)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": p99 * 1e3,
            "max_ms": float(lat.max() * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "p99_tail_arrivals_s": [float(tail.min()), float(tail.max())],
            "elements": int(elems), "span_s": float(span), "elements_per_s": float(elems / span)}
