"""ctypes binding of libmeshnbr.so (include/mesh_neighbors.h).

Argument marshalling only: every step of the neighbor pipelines runs in the
library's HIP kernels.  PyTorch provides device memory and the stream.  If the
library is missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import enum
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmeshnbr.so")

TRI3, TET4, HEX8 = 0, 1, 2
NODES_PER_ELEM = {TRI3: 3, TET4: 4, HEX8: 8}


class Status(enum.IntEnum):
    OK = 0
    INVALID_ARG = 1
    UNSUPPORTED_TYPE = 2
    WORKSPACE = 3
    CAPACITY = 4
    OVERFLOW = 5
    INDEX_RANGE = 6
    HIP = 7
    INTERNAL = 8


class MeshError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = Status(status)
        super().__init__(f"{where}: {status_string(status)} ({self.status.name})")


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


_lib = None

_c_i32, _c_i64, _c_sz, _c_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/mesh_neighbors.h
SIGNATURES = {
    "mesh_node_neighbors_query": (_c_i32, [_c_i64, _c_i32, _c_i32, ctypes.POINTER(_c_sz), ctypes.POINTER(_c_i64)]),
    "mesh_node_neighbors": (_c_i32, [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_sz, _c_p]),
    "mesh_elem_neighbors_query": (_c_i32, [_c_i64, _c_i32, _c_i32, ctypes.POINTER(_c_sz), ctypes.POINTER(_c_i64)]),
    "mesh_elem_neighbors": (_c_i32, [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_sz, _c_p]),
    "mesh_check": (_c_i32, [_c_p, _c_p]),
    "mesh_status_string": (ctypes.c_char_p, [_c_i32]),
    "mesh_abi_version": (_c_i32, []),
    "mesh_batch_node_neighbors_query": (_c_i32, [_c_i32, _c_i64, _c_i32, _c_i32, ctypes.POINTER(_c_sz),
                                                 ctypes.POINTER(_c_i64)]),
    "mesh_batch_node_neighbors": (_c_i32, [_c_p, _c_p, _c_i32, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p,
                                           _c_sz, _c_p]),
    "mesh_batch_elem_neighbors_query": (_c_i32, [_c_i32, _c_i64, _c_i32, ctypes.POINTER(_c_sz),
                                                 ctypes.POINTER(_c_i64)]),
    "mesh_batch_elem_neighbors": (_c_i32, [_c_p, _c_p, _c_i32, _c_i64, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_sz,
                                           _c_p]),
    "mesh_timing_enable": (_c_i32, [_c_i32]),
    "mesh_radix_shape_count": (_c_i32, []),
    "mesh_radix_shape_info": (_c_i32, [_c_i32, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "mesh_set_radix_shape": (_c_i32, [_c_i32]),
    "mesh_get_radix_shape": (_c_i32, []),
    "mesh_set_node_sort": (_c_i32, [_c_i32]),
    "mesh_get_node_sort": (_c_i32, []),
    "mesh_timing_read": (_c_i32, [ctypes.POINTER(KernelTime), _c_i32]),
    "mesh_graph_node_neighbors": (_c_i32, [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_sz,
                                           ctypes.POINTER(_c_p)]),
    "mesh_graph_elem_neighbors": (_c_i32, [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_sz,
                                           ctypes.POINTER(_c_p)]),
    "mesh_graph_batch_node_neighbors": (_c_i32, [_c_p, _c_p, _c_i32, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64,
                                                 _c_p, _c_sz, ctypes.POINTER(_c_p)]),
    "mesh_graph_batch_elem_neighbors": (_c_i32, [_c_p, _c_p, _c_i32, _c_i64, _c_i32, _c_p, _c_p, _c_i64, _c_p,
                                                 _c_sz, ctypes.POINTER(_c_p)]),
    "mesh_graph_launch": (_c_i32, [_c_p, _c_p]),
    "mesh_graph_destroy": (_c_i32, [_c_p]),
}


def lib() -> ctypes.CDLL:
    """Load libmeshnbr.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_04689_amd.build` "
                               "(the HIP library is required; there is no CPU path)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def status_string(status) -> str:
    return lib().mesh_status_string(int(status)).decode()


def radix_shapes():
    """[(threads per block, keys per thread)] of the radix tile shapes built in."""
    out = []
    for i in range(lib().mesh_radix_shape_count()):
        b, it = _c_i32(0), _c_i32(0)
        lib().mesh_radix_shape_info(i, ctypes.byref(b), ctypes.byref(it))
        out.append((b.value, it.value))
    return out


def set_radix_shape(shape: int = -1):
    """Select the radix tile shape for all later calls (-1 = default)."""
    st = lib().mesh_set_radix_shape(int(shape))
    if st != Status.OK:
        raise MeshError(st, "mesh_set_radix_shape")


def get_radix_shape() -> int:
    return int(lib().mesh_get_radix_shape())


NODE_SORT_FULL_KEY, NODE_SORT_VERTEX_ROWS, NODE_SORT_EDGE_ROWS = 0, 1, 2


def set_node_sort(mode: int):
    """Select the node algorithm of single meshes and batches (results are
    identical)."""
    st = lib().mesh_set_node_sort(int(mode))
    if st != Status.OK:
        raise MeshError(st, "mesh_set_node_sort")


def get_node_sort() -> int:
    return int(lib().mesh_get_node_sort())


def timing_enable(on: bool = True):
    """Record HIP-event durations of every library kernel launched from now on."""
    lib().mesh_timing_enable(1 if on else 0)


def timing_read():
    """{kernel name: (launches, total_ms, min_ms, max_ms)} since the last read (waits for them)."""
    buf = (KernelTime * 64)()
    n = lib().mesh_timing_read(buf, 64)
    if n < 0:
        raise RuntimeError("mesh_timing_read: event query failed")
    return {buf[i].name.decode(): (int(buf[i].launches), buf[i].total_ms, buf[i].min_ms, buf[i].max_ms)
            for i in range(min(n, 64))}


def _query(kind, n_elem, etype, n_vert):
    ws = _c_sz(0)
    cap = _c_i64(0)
    st = getattr(lib(), f"mesh_{kind}_neighbors_query")(int(n_elem), int(etype), int(n_vert),
                                                       ctypes.byref(ws), ctypes.byref(cap))
    if st != Status.OK:
        raise MeshError(st, f"mesh_{kind}_neighbors_query")
    return int(ws.value), int(cap.value)


def query_node(n_elem, etype, n_vert):
    """(workspace bytes, sufficient cols capacity) for the node relation."""
    return _query("node", n_elem, etype, n_vert)


def query_elem(n_elem, etype, n_vert):
    """(workspace bytes, sufficient cols capacity) for the element relation."""
    return _query("elem", n_elem, etype, n_vert)


def _stream_handle(stream, device):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


class NeighborBuild:
    """Device buffers for one relation ("node" or "elem") of one mesh shape.

    Allocates the workspace and outputs once; ``launch`` enqueues the
    pipeline on a stream without allocating or synchronising, ``result``
    checks the device error word and returns ``(row_ptr, cols[:nnz])``.
    """

    def __init__(self, kind, n_elem, etype, n_vert, device="cuda", cols_capacity=None):
        import torch

        if kind not in ("node", "elem"):
            raise ValueError(kind)
        self.kind = kind
        self.n_elem, self.etype, self.n_vert = int(n_elem), int(etype), int(n_vert)
        self.device = torch.device(device)
        ws_bytes, cap = _query(kind, n_elem, etype, n_vert)
        self.cols_capacity = int(cap if cols_capacity is None else cols_capacity)
        # 256-byte aligned workspace carved from a byte tensor
        self._ws_raw = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=self.device)
        pad = (-self._ws_raw.data_ptr()) % 256
        self.workspace = self._ws_raw[pad:pad + ws_bytes]
        self.ws_bytes = ws_bytes
        self.row_ptr = torch.empty(self.n_vert + 1, dtype=torch.int32, device=self.device)
        self.cols = torch.empty(max(self.cols_capacity, 1), dtype=torch.int32, device=self.device)
        self._fn = getattr(lib(), f"mesh_{kind}_neighbors")

    def launch(self, conn, stream=None, tuned=False):
        import torch

        if conn.device != self.device or conn.dtype != torch.int32 or not conn.is_contiguous():
            raise ValueError("conn must be a contiguous int32 tensor on the build's device")
        if tuned and self.etype in NODES_PER_ELEM:
            from . import autotune
            autotune.apply(self.kind, self.etype, self.n_elem)
        npe = NODES_PER_ELEM.get(self.etype)
        if npe is not None and conn.numel() != self.n_elem * npe:
            raise ValueError(f"conn has {conn.numel()} ids, expected {self.n_elem} x {npe}")
        st = self._fn(_ptr(conn), self.n_elem, self.etype, self.n_vert, _ptr(self.row_ptr),
                      _ptr(self.cols) if self.cols_capacity > 0 else ctypes.c_void_p(0), self.cols_capacity,
                      _ptr(self.workspace), self.ws_bytes, _stream_handle(stream, self.device))
        if st != Status.OK:
            raise MeshError(st, f"mesh_{self.kind}_neighbors")

    def check(self, stream=None):
        st = lib().mesh_check(_ptr(self.workspace), _stream_handle(stream, self.device))
        if st != Status.OK:
            raise MeshError(st, "mesh_check")

    def result(self, stream=None):
        self.check(stream)
        nnz = int(self.row_ptr[-1].item())
        return self.row_ptr, self.cols[:nnz]

    def capture(self, conn, tuned=False):
        """A Graph replaying ``launch(conn)`` on this build's buffers; conn's
        contents may change between replays, its address and size may not."""
        import torch

        if conn.device != self.device or conn.dtype != torch.int32 or not conn.is_contiguous():
            raise ValueError("conn must be a contiguous int32 tensor on the build's device")
        if tuned and self.etype in NODES_PER_ELEM:
            from . import autotune
            autotune.apply(self.kind, self.etype, self.n_elem)
        npe = NODES_PER_ELEM.get(self.etype)
        if npe is not None and conn.numel() != self.n_elem * npe:
            raise ValueError(f"conn has {conn.numel()} ids, expected {self.n_elem} x {npe}")
        h = _c_p()
        with _device_guard(self.device):
            st = getattr(lib(), f"mesh_graph_{self.kind}_neighbors")(
                _ptr(conn), self.n_elem, self.etype, self.n_vert, _ptr(self.row_ptr),
                _ptr(self.cols) if self.cols_capacity > 0 else ctypes.c_void_p(0), self.cols_capacity,
                _ptr(self.workspace), self.ws_bytes, ctypes.byref(h))
        if st != Status.OK:
            raise MeshError(st, f"mesh_graph_{self.kind}_neighbors")
        return Graph(h, self.device, keep=(conn, self._ws_raw, self.row_ptr, self.cols))


class Graph:
    """An instantiated HIP graph of one call (see mesh_graph_* in the
    header).  Holds references to the buffers it was captured on."""

    def __init__(self, handle, device, keep=()):
        self._h = handle
        self.device = device
        self._keep = keep

    def launch(self, stream=None):
        if not self._h:
            raise ValueError("graph was destroyed")
        st = lib().mesh_graph_launch(self._h, _stream_handle(stream, self.device))
        if st != Status.OK:
            raise MeshError(st, "mesh_graph_launch")

    def destroy(self):
        if self._h:
            lib().mesh_graph_destroy(self._h)
            self._h = None
            self._keep = ()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _device_guard(device):
    import torch

    return torch.cuda.device(device)


def _n_elem(conn, etype):
    if conn.dim() == 2:
        return conn.shape[0]
    return conn.numel() // NODES_PER_ELEM.get(int(etype), 1)


def node_neighbors(conn, etype, n_vert, stream=None):
    """One-ring neighboring nodes of every vertex: (row_ptr, cols) on conn's device."""
    b = NeighborBuild("node", _n_elem(conn, etype), etype, n_vert, conn.device)
    b.launch(conn, stream)
    return b.result(stream)


def elem_neighbors(conn, etype, n_vert, stream=None):
    """One-ring neighboring elements of every vertex: (row_ptr, cols) on conn's device."""
    b = NeighborBuild("elem", _n_elem(conn, etype), etype, n_vert, conn.device)
    b.launch(conn, stream)
    return b.result(stream)


# ---------------------------------------------------------------------------
# Batches of meshes
# ---------------------------------------------------------------------------

EDGES_PER_ELEM = {TRI3: 3, TET4: 6, HEX8: 12}


def segment_table(meshes, conn_offs=None):
    """mesh_segment records (numpy structured array, 48 bytes each) for a
    list of (n_elem, etype, n_vert), plus the totals (pairs, slots, vertices,
    ids).  The meshes' ids lie back to back in one shared connectivity array,
    or, with ``conn_offs``, mesh m's ids start at index conn_offs[m] of it;
    ``ids`` is then the end of the furthest mesh."""
    import numpy as np

    dt = np.dtype([("conn_off", "<i8"), ("n_elem", "<i8"), ("pair_off", "<i8"), ("slot_off", "<i8"),
                   ("vert_off", "<i4"), ("n_vert", "<i4"), ("etype", "<i4"), ("reserved", "<i4")])
    assert dt.itemsize == 48
    seg = np.zeros(len(meshes), dtype=dt)
    conn_off = pair_off = slot_off = vert_off = 0
    ids_end = 0
    for i, (n_elem, etype, n_vert) in enumerate(meshes):
        npe, ne = NODES_PER_ELEM[int(etype)], EDGES_PER_ELEM[int(etype)]
        if conn_offs is not None:
            conn_off = int(conn_offs[i])
        seg[i] = (conn_off, n_elem, pair_off, slot_off, vert_off, n_vert, etype, 0)
        conn_off += npe * n_elem
        ids_end = max(ids_end, conn_off)
        pair_off += 2 * ne * n_elem
        slot_off += npe * n_elem
        vert_off += n_vert
    return seg, {"pairs": pair_off, "slots": slot_off, "vert": vert_off, "ids": ids_end,
                 "max_vert": max([int(m[2]) for m in meshes], default=0)}


class BatchBuild:
    """Device buffers for one relation ("node" or "elem") of a batch of meshes.

    ``meshes`` is a list of (n_elem, etype, n_vert); the connectivity passed to
    ``launch`` is all meshes' int32 ids back to back, each mesh's ids local.
    ``result`` gives the global CSR (cols in local ids); ``mesh_csr(m)`` the
    slice of mesh m rebased to start at 0.  ``reset(meshes)`` re-targets the
    build at another batch, reusing its device buffers when they are large
    enough (they only grow)."""

    def __init__(self, kind, meshes, device="cuda", conn_offs=None):
        import torch

        if kind not in ("node", "elem"):
            raise ValueError(kind)
        self.kind = kind
        self.device = torch.device(device)
        self._ws_raw = self._rp = self._cols = self._segs = None
        self._seg_pinned = self._seg_event = None
        self.reset(meshes, conn_offs=conn_offs)

    def reset(self, meshes, stream=None, conn_offs=None):
        """Re-target at another batch.  The segment table is uploaded
        asynchronously on ``stream`` (default: the current stream), so reset
        and launch must use the same stream.  ``conn_offs`` places each mesh's
        ids in the connectivity passed to launch (default: back to back)."""
        import contextlib

        import torch

        seg, tot = segment_table(meshes, conn_offs)
        self.custom_offsets = conn_offs is not None
        self.seg_host = seg
        self.totals = tot
        self.n_mesh = len(meshes)
        ws, cap = _c_sz(0), _c_i64(0)
        if self.kind == "node":
            st = lib().mesh_batch_node_neighbors_query(self.n_mesh, tot["pairs"], tot["vert"], tot["max_vert"],
                                                       ctypes.byref(ws), ctypes.byref(cap))
        else:
            st = lib().mesh_batch_elem_neighbors_query(self.n_mesh, tot["slots"], tot["vert"], ctypes.byref(ws),
                                                       ctypes.byref(cap))
        if st != Status.OK:
            raise MeshError(st, f"mesh_batch_{self.kind}_neighbors_query")
        self.ws_bytes = int(ws.value)
        self.cols_capacity = int(cap.value)

        def grow(buf, n, dtype):
            if buf is None or buf.numel() < n:
                return torch.empty(max(n, 1), dtype=dtype, device=self.device)
            return buf

        self._ws_raw = grow(self._ws_raw, self.ws_bytes + 256, torch.uint8)
        pad = (-self._ws_raw.data_ptr()) % 256
        self.workspace = self._ws_raw[pad:pad + self.ws_bytes]
        self._rp = grow(self._rp, tot["vert"] + 1, torch.int32)
        self.row_ptr = self._rp[:tot["vert"] + 1]
        self._cols = grow(self._cols, self.cols_capacity, torch.int32)
        self.cols = self._cols
        nbytes = 48 * len(meshes)
        self._segs = grow(self._segs, max(nbytes, 1), torch.uint8)
        if nbytes:
            # the pinned staging buffer is rewritten only after its previous upload has completed
            if self._seg_event is not None:
                self._seg_event.synchronize()
            if self._seg_pinned is None or self._seg_pinned.numel() < nbytes:
                self._seg_pinned = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
            self._seg_pinned[:nbytes].numpy()[:] = seg.view("u1")
            ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
            with ctx:
                self._segs[:nbytes].copy_(self._seg_pinned[:nbytes], non_blocking=True)
                self._seg_event = torch.cuda.Event()
                self._seg_event.record()
        self.segs = self._segs

    def launch(self, conn, stream=None, tuned=False):
        import torch

        if conn.device != self.device or conn.dtype != torch.int32 or not conn.is_contiguous():
            raise ValueError("conn must be a contiguous int32 tensor on the build's device")
        if tuned:
            from . import autotune
            autotune.apply_batch(self.kind, self.totals["pairs"] if self.kind == "node" else self.totals["slots"])
        self._check_conn(conn)
        t = self.totals
        if self.kind == "node":
            st = lib().mesh_batch_node_neighbors(_ptr(conn), _ptr(self.segs), self.n_mesh, t["pairs"], t["vert"],
                                                 t["max_vert"], _ptr(self.row_ptr), _ptr(self.cols),
                                                 self.cols_capacity, _ptr(self.workspace), self.ws_bytes,
                                                 _stream_handle(stream, self.device))
        else:
            st = lib().mesh_batch_elem_neighbors(_ptr(conn), _ptr(self.segs), self.n_mesh, t["slots"], t["vert"],
                                                 _ptr(self.row_ptr), _ptr(self.cols), self.cols_capacity,
                                                 _ptr(self.workspace), self.ws_bytes,
                                                 _stream_handle(stream, self.device))
        if st != Status.OK:
            raise MeshError(st, f"mesh_batch_{self.kind}_neighbors")

    def _check_conn(self, conn):
        need = self.totals["ids"]
        if (conn.numel() < need) if self.custom_offsets else (conn.numel() != need):
            raise ValueError(f"conn has {conn.numel()} ids, the segments cover {need}")

    def check(self, stream=None):
        st = lib().mesh_check(_ptr(self.workspace), _stream_handle(stream, self.device))
        if st != Status.OK:
            raise MeshError(st, "mesh_check")

    def result(self, stream=None):
        self.check(stream)
        nnz = int(self.row_ptr[-1].item())
        return self.row_ptr, self.cols[:nnz]

    def capture(self, conn, tuned=False):
        """A Graph replaying ``launch(conn)`` for the current batch layout
        (totals fixed; conn and segment contents may change between replays
        as long as the totals stay the same)."""
        import torch

        if conn.device != self.device or conn.dtype != torch.int32 or not conn.is_contiguous():
            raise ValueError("conn must be a contiguous int32 tensor on the build's device")
        if tuned:
            from . import autotune
            autotune.apply_batch(self.kind, self.totals["pairs"] if self.kind == "node" else self.totals["slots"])
        self._check_conn(conn)
        t = self.totals
        h = _c_p()
        with _device_guard(self.device):
            if self.kind == "node":
                st = lib().mesh_graph_batch_node_neighbors(_ptr(conn), _ptr(self.segs), self.n_mesh, t["pairs"],
                                                           t["vert"], t["max_vert"], _ptr(self.row_ptr),
                                                           _ptr(self.cols), self.cols_capacity, _ptr(self.workspace),
                                                           self.ws_bytes, ctypes.byref(h))
            else:
                st = lib().mesh_graph_batch_elem_neighbors(_ptr(conn), _ptr(self.segs), self.n_mesh, t["slots"],
                                                           t["vert"], _ptr(self.row_ptr), _ptr(self.cols),
                                                           self.cols_capacity, _ptr(self.workspace), self.ws_bytes,
                                                           ctypes.byref(h))
        if st != Status.OK:
            raise MeshError(st, f"mesh_graph_batch_{self.kind}_neighbors")
        # the graph holds the buffers themselves: a later reset() may replace them
        return Graph(h, self.device, keep=(conn, self._ws_raw, self._rp, self._cols, self._segs))

    def mesh_csr(self, m, row_ptr_host=None):
        """(row_ptr, cols) of mesh m alone, as device tensors, after result()."""
        seg = self.seg_host[m]
        v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
        rp = self.row_ptr[v0:v0 + nv + 1]
        if row_ptr_host is not None:
            a, b = int(row_ptr_host[v0]), int(row_ptr_host[v0 + nv])
        else:
            a, b = int(rp[0].item()), int(rp[-1].item())
        return rp - a, self.cols[a:b]


def concat_conn(conns):
    """One int32 array holding the connectivities back to back (row-major)."""
    import numpy as np

    if not conns:
        return np.zeros(0, dtype=np.int32)
    return np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.int32).ravel() for c in conns]))
