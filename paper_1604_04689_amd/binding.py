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

TRI3, TET4, HEX8, QUAD4, WEDGE6, PYRAMID5 = 0, 1, 2, 3, 4, 5
NODES_PER_ELEM = {TRI3: 3, TET4: 4, HEX8: 8, QUAD4: 4, WEDGE6: 6, PYRAMID5: 5}
EDGES_PER_ELEM = {TRI3: 3, TET4: 6, HEX8: 12, QUAD4: 4, WEDGE6: 9, PYRAMID5: 8}


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
    SCRATCH_LIMIT = 9
    CHUNK = 10


class MeshError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = Status(status)
        super().__init__(f"{where}: {status_string(status)} ({self.status.name})")


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


NODE_SORT_FULL_KEY, NODE_SORT_VERTEX_ROWS, NODE_SORT_EDGE_ROWS, NODE_SORT_ELEM_ROWS = 0, 1, 2, 3
NODE_SORT_NAMES = {0: "full_key", 1: "vertex_rows", 2: "edge_rows", 3: "elem_rows"}


class Options(ctypes.Structure):
    """mesh_options: per-call choices that never change results (-1 =
    library default): node algorithm, radix tile shape, digit width, and
    chunk_keys, the pair budget of a bounded-memory build (-1 or 0: the whole
    mesh at once)."""
    _fields_ = [("node_sort", ctypes.c_int32), ("radix_shape", ctypes.c_int32), ("digit_bits", ctypes.c_int32),
                ("chunk_keys", ctypes.c_int32), ("reserved", ctypes.c_int32 * 4)]

    def as_dict(self):
        return {"node_sort": int(self.node_sort), "radix_shape": int(self.radix_shape),
                "digit_bits": int(self.digit_bits), "chunk_keys": int(self.chunk_keys)}


OPTION_KEYS = ("node_sort", "radix_shape", "digit_bits", "chunk_keys")


def make_options(options=None) -> Options:
    """Options from None (defaults), an Options, or a dict with any of
    node_sort, radix_shape, digit_bits, chunk_keys."""
    if isinstance(options, Options):
        return options
    o = Options(-1, -1, -1, -1)
    for k, v in (options or {}).items():
        if k not in OPTION_KEYS:
            raise ValueError(f"unknown option {k}")
        setattr(o, k, -1 if v is None else int(v))
    return o


_lib = None

_c_i32, _c_i64, _c_sz, _c_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
_P_SZ, _P_I64, _P_I32, _P_P = (ctypes.POINTER(_c_sz), ctypes.POINTER(_c_i64), ctypes.POINTER(_c_i32),
                               ctypes.POINTER(_c_p))
_P_OPT = ctypes.POINTER(Options)

# name -> (restype, argtypes); mirrors include/mesh_neighbors.h
_ONE = [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _P_OPT, _c_p, _c_sz]
_BOTH = [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_p, _c_i64, _P_OPT, _c_p, _c_sz]
_BNODE = [_c_p, _c_p, _c_i32, _c_i64, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _P_OPT, _c_p, _c_sz]
_BELEM = [_c_p, _c_p, _c_i32, _c_i64, _c_i32, _c_p, _c_p, _c_i64, _P_OPT, _c_p, _c_sz]
_BBOTH = [_c_p, _c_p, _c_i32, _c_i64, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_p, _c_i64, _P_OPT,
          _c_p, _c_sz]
SIGNATURES = {
    "mesh_default_options": (Options, []),
    "mesh_node_neighbors_query": (_c_i32, [_c_i64, _c_i32, _c_i32, _P_OPT, _P_SZ, _P_I64]),
    "mesh_node_neighbors": (_c_i32, _ONE + [_c_p]),
    "mesh_elem_neighbors_query": (_c_i32, [_c_i64, _c_i32, _c_i32, _P_OPT, _P_SZ, _P_I64]),
    "mesh_elem_neighbors": (_c_i32, _ONE + [_c_p]),
    "mesh_neighbors_query": (_c_i32, [_c_i64, _c_i32, _c_i32, _P_OPT, _P_SZ, _P_I64, _P_I64]),
    "mesh_neighbors": (_c_i32, _BOTH + [_c_p]),
    "mesh_neighbors_noalloc": (_c_i32, [_c_p, _c_i64, _c_i32, _c_i32, _c_p, _c_p, _c_i64, _c_p, _c_p, _c_i64, _P_OPT,
                                        _c_p]),
    "mesh_mixed_neighbors_query": (_c_i32, [_c_i64, _c_i64, _c_i64, _c_i32, _P_OPT, _P_SZ, _P_I64, _P_I64]),
    "mesh_mixed_neighbors": (_c_i32, [_c_p, _c_p, _c_p, _c_i64, _c_i64, _c_i64, _c_i32, _c_p, _c_p, _c_i64, _c_p,
                                      _c_p, _c_i64, _P_OPT, _c_p, _c_sz, _c_p]),
    "mesh_batch_node_neighbors_query": (_c_i32, [_c_i32, _c_i64, _c_i64, _c_i32, _c_i32, _P_OPT, _P_SZ, _P_I64]),
    "mesh_batch_node_neighbors": (_c_i32, _BNODE + [_c_p]),
    "mesh_batch_elem_neighbors_query": (_c_i32, [_c_i32, _c_i64, _c_i32, _P_OPT, _P_SZ, _P_I64]),
    "mesh_batch_elem_neighbors": (_c_i32, _BELEM + [_c_p]),
    "mesh_batch_neighbors_query": (_c_i32, [_c_i32, _c_i64, _c_i64, _c_i32, _c_i32, _P_OPT, _P_SZ, _P_I64,
                                            _P_I64]),
    "mesh_batch_neighbors": (_c_i32, _BBOTH + [_c_p]),
    "mesh_graph_node_neighbors": (_c_i32, _ONE + [_P_P]),
    "mesh_graph_elem_neighbors": (_c_i32, _ONE + [_P_P]),
    "mesh_graph_neighbors": (_c_i32, _BOTH + [_P_P]),
    "mesh_graph_batch_node_neighbors": (_c_i32, _BNODE + [_P_P]),
    "mesh_graph_batch_elem_neighbors": (_c_i32, _BELEM + [_P_P]),
    "mesh_graph_batch_neighbors": (_c_i32, _BBOTH + [_P_P]),
    "mesh_graph_launch": (_c_i32, [_c_p, _c_p]),
    "mesh_graph_destroy": (_c_i32, [_c_p]),
    "mesh_check": (_c_i32, [_c_p, _c_p]),
    "mesh_status_string": (ctypes.c_char_p, [_c_i32]),
    "mesh_abi_version": (_c_i32, []),
    "mesh_radix_shape_count": (_c_i32, []),
    "mesh_radix_shape_info": (_c_i32, [_c_i32, _P_I32, _P_I32]),
    "mesh_radix_launch_shape": (_c_i32, [_c_i32, _c_i32, _c_i64, _P_I32, _P_I32, _P_I32]),
    "mesh_timing_enable": (_c_i32, [_c_i32]),
    "mesh_timing_read": (_c_i32, [ctypes.POINTER(KernelTime), _c_i32]),
    "mesh_timing_select": (_c_i32, [ctypes.c_char_p]),
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


def radix_launch_shape(shape, digit_bits, n_keys):
    """(block, items, digit bits) a pass over n_keys keys launches with when
    the options ask for `shape` and `digit_bits` (-1: defaults)."""
    b, it, bits = _c_i32(0), _c_i32(0), _c_i32(0)
    st = lib().mesh_radix_launch_shape(int(shape), int(digit_bits), int(n_keys), ctypes.byref(b), ctypes.byref(it),
                                       ctypes.byref(bits))
    if st != Status.OK:
        raise MeshError(st, "mesh_radix_launch_shape")
    return b.value, it.value, bits.value


def timing_enable(on: bool = True):
    """Record HIP-event durations of every library kernel launched from now on."""
    lib().mesh_timing_enable(1 if on else 0)


def timing_select(names=None):
    """Time only the launches with these names (an iterable of launch names
    as timing_read reports them); None or empty: every launch."""
    s = ",".join(names) if names else ""
    _check(lib().mesh_timing_select(s.encode()), "mesh_timing_select")


def timing_read():
    """{kernel name: (launches, total_ms, min_ms, max_ms)} since the last read (waits for them)."""
    buf = (KernelTime * 64)()
    n = lib().mesh_timing_read(buf, 64)
    if n < 0:
        raise RuntimeError("mesh_timing_read: event query failed")
    return {buf[i].name.decode(): (int(buf[i].launches), buf[i].total_ms, buf[i].min_ms, buf[i].max_ms)
            for i in range(min(n, 64))}


def _check(st, where):
    if st != Status.OK:
        raise MeshError(st, where)


def query(kind, n_elem, etype, n_vert, options=None):
    """(workspace bytes, cols capacity) for kind "node" or "elem", or
    (workspace bytes, node capacity, elem capacity) for "both"."""
    o = make_options(options)
    ws, cap, cap2 = _c_sz(0), _c_i64(0), _c_i64(0)
    if kind == "both":
        _check(lib().mesh_neighbors_query(int(n_elem), int(etype), int(n_vert), ctypes.byref(o), ctypes.byref(ws),
                                          ctypes.byref(cap), ctypes.byref(cap2)), "mesh_neighbors_query")
        return int(ws.value), int(cap.value), int(cap2.value)
    fn = getattr(lib(), f"mesh_{kind}_neighbors_query")
    _check(fn(int(n_elem), int(etype), int(n_vert), ctypes.byref(o), ctypes.byref(ws), ctypes.byref(cap)),
           f"mesh_{kind}_neighbors_query")
    return int(ws.value), int(cap.value)


def query_node(n_elem, etype, n_vert, options=None):
    """(workspace bytes, sufficient cols capacity) for the node relation."""
    return query("node", n_elem, etype, n_vert, options)


def query_elem(n_elem, etype, n_vert, options=None):
    """(workspace bytes, sufficient cols capacity) for the element relation."""
    return query("elem", n_elem, etype, n_vert, options)


def _stream_handle(stream, device):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _workspace(torch, nbytes, device, old=None):
    """A 256-byte aligned byte view of at least nbytes (reusing `old`'s
    storage when it is large enough): (raw tensor, aligned view)."""
    raw = old if old is not None and old.numel() >= nbytes + 256 else \
        torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    pad = (-raw.data_ptr()) % 256
    return raw, raw[pad:pad + nbytes]


def _resolve(kind, etype, n_elem, options):
    """Options for a build: "tuned" looks them up in the tuning table."""
    if isinstance(options, str):
        if options != "tuned":
            raise ValueError(options)
        from . import autotune
        return make_options(autotune.options_for(kind, etype, n_elem))
    return make_options(options)


def _check_conn(torch, conn, device):
    if conn.device != device or conn.dtype != torch.int32 or not conn.is_contiguous():
        raise ValueError("conn must be a contiguous int32 tensor on the build's device")


class NeighborBuild:
    """Device buffers for one mesh shape and one relation: kind "node",
    "elem", or "both" (one call building both).

    The options (None: library defaults; a dict; "tuned": from the tuning
    table) are fixed here, since the workspace size depends on them.
    ``launch`` enqueues the pipeline on a stream without allocating or
    synchronising; ``result`` checks the device error word and returns
    ``(row_ptr, cols[:nnz])`` (for "both": ``((node row_ptr, cols), (elem
    row_ptr, cols))``).
    """

    def __init__(self, kind, n_elem, etype, n_vert, device="cuda", cols_capacity=None, options=None):
        import torch

        if kind not in ("node", "elem", "both"):
            raise ValueError(kind)
        self.kind = kind
        self.n_elem, self.etype, self.n_vert = int(n_elem), int(etype), int(n_vert)
        self.device = torch.device(device)
        self.options = _resolve(kind, etype, n_elem, options)
        q = query(kind, n_elem, etype, n_vert, self.options)
        ws_bytes = q[0]
        self.cols_capacity = int(q[1] if cols_capacity is None else cols_capacity)
        self._ws_raw, self.workspace = _workspace(torch, ws_bytes, self.device)
        self.ws_bytes = ws_bytes
        self.row_ptr = torch.empty(self.n_vert + 1, dtype=torch.int32, device=self.device)
        self.cols = torch.empty(max(self.cols_capacity, 1), dtype=torch.int32, device=self.device)
        if kind == "both":
            self.elem_capacity = int(q[2])
            self.elem_row_ptr = torch.empty(self.n_vert + 1, dtype=torch.int32, device=self.device)
            self.elem_cols = torch.empty(max(self.elem_capacity, 1), dtype=torch.int32, device=self.device)

    def _args(self, conn):
        a = [_ptr(conn), self.n_elem, self.etype, self.n_vert, _ptr(self.row_ptr),
             _ptr(self.cols) if self.cols_capacity > 0 else ctypes.c_void_p(0), self.cols_capacity]
        if self.kind == "both":
            a += [_ptr(self.elem_row_ptr), _ptr(self.elem_cols) if self.elem_capacity > 0 else ctypes.c_void_p(0),
                  self.elem_capacity]
        return a + [ctypes.byref(self.options), _ptr(self.workspace), self.ws_bytes]

    def _name(self, prefix="mesh_"):
        return prefix + ("neighbors" if self.kind == "both" else f"{self.kind}_neighbors")

    def _validate(self, conn):
        import torch

        _check_conn(torch, conn, self.device)
        npe = NODES_PER_ELEM.get(self.etype)
        if npe is not None and conn.numel() != self.n_elem * npe:
            raise ValueError(f"conn has {conn.numel()} ids, expected {self.n_elem} x {npe}")

    def launch(self, conn, stream=None):
        self._validate(conn)
        name = self._name()
        _check(getattr(lib(), name)(*self._args(conn), _stream_handle(stream, self.device)), name)

    def check(self, stream=None):
        _check(lib().mesh_check(_ptr(self.workspace), _stream_handle(stream, self.device)), "mesh_check")

    def result(self, stream=None):
        self.check(stream)
        nnz = int(self.row_ptr[-1].item())
        if self.kind == "both":
            enz = int(self.elem_row_ptr[-1].item())
            return (self.row_ptr, self.cols[:nnz]), (self.elem_row_ptr, self.elem_cols[:enz])
        return self.row_ptr, self.cols[:nnz]

    def capture(self, conn):
        """A Graph replaying ``launch(conn)`` on this build's buffers; conn's
        contents may change between replays, its address and size may not."""
        self._validate(conn)
        h = _c_p()
        name = self._name("mesh_graph_")
        with _device_guard(self.device):
            st = getattr(lib(), name)(*self._args(conn), ctypes.byref(h))
        _check(st, name)
        keep = (conn, self._ws_raw, self.row_ptr, self.cols) + (
            (self.elem_row_ptr, self.elem_cols) if self.kind == "both" else ())
        return Graph(h, self.device, keep=keep)


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
        _check(lib().mesh_graph_launch(self._h, _stream_handle(stream, self.device)), "mesh_graph_launch")

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


def node_neighbors(conn, etype, n_vert, stream=None, options=None):
    """One-ring neighboring nodes of every vertex: (row_ptr, cols) on conn's device."""
    b = NeighborBuild("node", _n_elem(conn, etype), etype, n_vert, conn.device, options=options)
    b.launch(conn, stream)
    return b.result(stream)


def elem_neighbors(conn, etype, n_vert, stream=None, options=None):
    """One-ring neighboring elements of every vertex: (row_ptr, cols) on conn's device."""
    b = NeighborBuild("elem", _n_elem(conn, etype), etype, n_vert, conn.device, options=options)
    b.launch(conn, stream)
    return b.result(stream)


def neighbors(conn, etype, n_vert, stream=None, options=None):
    """Both relations in one call: ((node row_ptr, cols), (elem row_ptr, cols))."""
    b = NeighborBuild("both", _n_elem(conn, etype), etype, n_vert, conn.device, options=options)
    b.launch(conn, stream)
    return b.result(stream)


NOALLOC_SCRATCH_BYTES = 64 << 20  # MESH_NOALLOC_SCRATCH_BYTES


def neighbors_noalloc(conn, etype, n_vert, out, stream=None, options=None, check=True):
    """Both relations through mesh_neighbors_noalloc: no workspace, the
    library's fixed scratch array instead.  ``out`` = (node_row_ptr,
    node_cols, elem_row_ptr, elem_cols), int32 tensors on conn's device that
    the caller owns (row_ptr n_vert + 1 entries; cols capacities from
    ``query("both", ...)``).  With check=True the device error word is read
    (mesh_check(NULL)) and ((node row_ptr, cols[:nnz]), (elem row_ptr,
    cols[:nnz])) returned; else nothing is synchronised and None returned."""
    import torch

    _check_conn(torch, conn, conn.device)
    n_elem = _n_elem(conn, etype)
    nrp, ncols, erp, ecols = out
    for t in out:
        if t.device != conn.device or t.dtype != torch.int32 or not t.is_contiguous():
            raise ValueError("outputs must be contiguous int32 tensors on conn's device")
    if nrp.numel() != int(n_vert) + 1 or erp.numel() != int(n_vert) + 1:
        raise ValueError("row_ptr outputs need n_vert + 1 entries")
    o = make_options(options)
    h = _stream_handle(stream, conn.device)
    with _device_guard(conn.device):
        _check(lib().mesh_neighbors_noalloc(_ptr(conn), int(n_elem), int(etype), int(n_vert), _ptr(nrp),
                                            _ptr(ncols) if ncols.numel() else ctypes.c_void_p(0), ncols.numel(),
                                            _ptr(erp), _ptr(ecols) if ecols.numel() else ctypes.c_void_p(0),
                                            ecols.numel(), ctypes.byref(o), h), "mesh_neighbors_noalloc")
        if not check:
            return None
        _check(lib().mesh_check(None, h), "mesh_check")
    nnz, enz = int(nrp[-1].item()), int(erp[-1].item())
    return (nrp, ncols[:nnz]), (erp, ecols[:enz])


# ---------------------------------------------------------------------------
# Meshes of several element types
# ---------------------------------------------------------------------------

def mixed_layout(etypes):
    """(elem_off int32 [n+1], n_ids, n_pairs) of elements of the given types,
    their ids back to back."""
    import numpy as np

    et = np.asarray(etypes, dtype=np.int64)
    npe = np.array([NODES_PER_ELEM[t] for t in range(6)], dtype=np.int64)[et]
    nedge = np.array([EDGES_PER_ELEM[t] for t in range(6)], dtype=np.int64)[et]
    off = np.zeros(et.size + 1, dtype=np.int64)
    np.cumsum(npe, out=off[1:])
    return off.astype(np.int32), int(off[-1]), int(2 * nedge.sum())


class MixedBuild:
    """Both relations of a mesh whose elements carry their own types
    (mesh_mixed_neighbors).  The node relation takes the ELEM_ROWS algorithm."""

    def __init__(self, n_elem, n_ids, n_pairs, n_vert, device="cuda", options=None):
        import torch

        self.n_elem, self.n_ids, self.n_pairs, self.n_vert = int(n_elem), int(n_ids), int(n_pairs), int(n_vert)
        self.device = torch.device(device)
        self.options = make_options(options)
        ws, c1, c2 = _c_sz(0), _c_i64(0), _c_i64(0)
        _check(lib().mesh_mixed_neighbors_query(self.n_elem, self.n_ids, self.n_pairs, self.n_vert,
                                                ctypes.byref(self.options), ctypes.byref(ws), ctypes.byref(c1),
                                                ctypes.byref(c2)), "mesh_mixed_neighbors_query")
        self.ws_bytes = int(ws.value)
        self.node_capacity, self.elem_capacity = int(c1.value), int(c2.value)
        self._ws_raw, self.workspace = _workspace(torch, self.ws_bytes, self.device)
        self.row_ptr = torch.empty(self.n_vert + 1, dtype=torch.int32, device=self.device)
        self.cols = torch.empty(max(self.node_capacity, 1), dtype=torch.int32, device=self.device)
        self.elem_row_ptr = torch.empty(self.n_vert + 1, dtype=torch.int32, device=self.device)
        self.elem_cols = torch.empty(max(self.elem_capacity, 1), dtype=torch.int32, device=self.device)

    def launch(self, conn, elem_off, etypes, stream=None):
        import torch

        _check_conn(torch, conn, self.device)
        _check_conn(torch, elem_off, self.device)
        if etypes.device != self.device or etypes.dtype != torch.uint8 or not etypes.is_contiguous():
            raise ValueError("etypes must be a contiguous uint8 tensor on the build's device")
        if elem_off.numel() != self.n_elem + 1 or etypes.numel() != self.n_elem or conn.numel() < self.n_ids:
            raise ValueError("elem_off, etypes or conn do not match the build's sizes")
        _check(lib().mesh_mixed_neighbors(
            _ptr(conn), _ptr(elem_off), _ptr(etypes), self.n_elem, self.n_ids, self.n_pairs, self.n_vert,
            _ptr(self.row_ptr), _ptr(self.cols) if self.node_capacity > 0 else ctypes.c_void_p(0),
            self.node_capacity, _ptr(self.elem_row_ptr),
            _ptr(self.elem_cols) if self.elem_capacity > 0 else ctypes.c_void_p(0), self.elem_capacity,
            ctypes.byref(self.options), _ptr(self.workspace), self.ws_bytes, _stream_handle(stream, self.device)),
            "mesh_mixed_neighbors")

    def check(self, stream=None):
        _check(lib().mesh_check(_ptr(self.workspace), _stream_handle(stream, self.device)), "mesh_check")

    def result(self, stream=None):
        self.check(stream)
        nnz, enz = int(self.row_ptr[-1].item()), int(self.elem_row_ptr[-1].item())
        return (self.row_ptr, self.cols[:nnz]), (self.elem_row_ptr, self.elem_cols[:enz])


def mixed_neighbors(conn, etypes, n_vert, stream=None, options=None):
    """Both relations of a mixed mesh given as flat int32 ids (device tensor)
    and per-element type codes (device uint8 tensor)."""
    import torch

    elem_off, n_ids, n_pairs = mixed_layout(etypes.cpu().numpy())
    b = MixedBuild(etypes.numel(), n_ids, n_pairs, n_vert, conn.device, options=options)
    b.launch(conn, torch.as_tensor(elem_off).to(conn.device), etypes, stream)
    return b.result(stream)


# ---------------------------------------------------------------------------
# Batches of meshes
# ---------------------------------------------------------------------------

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
    """Device buffers for one relation ("node", "elem" or "both") of a batch
    of meshes.

    ``meshes`` is a list of (n_elem, etype, n_vert); the connectivity passed to
    ``launch`` is all meshes' int32 ids back to back, each mesh's ids local.
    ``result`` gives the global CSR (cols in local ids); ``mesh_csr(m)`` the
    slice of mesh m rebased to start at 0.  ``reset(meshes)`` re-targets the
    build at another batch, reusing its device buffers when they are large
    enough (they only grow).  Options are fixed at construction ("tuned":
    from the tuning table's batch entries)."""

    def __init__(self, kind, meshes, device="cuda", conn_offs=None, options=None):
        import torch

        if kind not in ("node", "elem", "both"):
            raise ValueError(kind)
        self.kind = kind
        self.device = torch.device(device)
        self._tuned = isinstance(options, str)
        if self._tuned and options != "tuned":
            raise ValueError(options)
        self._options_arg = None if self._tuned else make_options(options)
        self._ws_raw = self._rp = self._cols = self._erp = self._ecols = self._segs = None
        self._seg_pinned = self._seg_event = None
        self.reset(meshes, conn_offs=conn_offs)

    def reset(self, meshes, stream=None, conn_offs=None, outputs=True):
        """Re-target at another batch.  The segment table is uploaded
        asynchronously on ``stream`` (default: the current stream), so reset
        and launch must use the same stream.  ``conn_offs`` places each mesh's
        ids in the connectivity passed to launch (default: back to back).
        outputs=False leaves the outputs to the caller (set_outputs)."""
        import contextlib

        import torch

        seg, tot = segment_table(meshes, conn_offs)
        self.custom_offsets = conn_offs is not None
        self.seg_host = seg
        self.totals = tot
        self.n_mesh = len(meshes)
        if self._tuned:
            from . import autotune
            self.options = make_options(autotune.batch_options_for(self.kind, tot["pairs"], tot["slots"]))
        else:
            self.options = self._options_arg
        ws, cap, cap2 = _c_sz(0), _c_i64(0), _c_i64(0)
        o = ctypes.byref(self.options)
        if self.kind == "node":
            _check(lib().mesh_batch_node_neighbors_query(self.n_mesh, tot["pairs"], tot["slots"], tot["vert"],
                                                         tot["max_vert"], o, ctypes.byref(ws), ctypes.byref(cap)),
                   "mesh_batch_node_neighbors_query")
        elif self.kind == "elem":
            _check(lib().mesh_batch_elem_neighbors_query(self.n_mesh, tot["slots"], tot["vert"], o, ctypes.byref(ws),
                                                         ctypes.byref(cap)), "mesh_batch_elem_neighbors_query")
        else:
            _check(lib().mesh_batch_neighbors_query(self.n_mesh, tot["pairs"], tot["slots"], tot["vert"],
                                                    tot["max_vert"], o, ctypes.byref(ws), ctypes.byref(cap),
                                                    ctypes.byref(cap2)), "mesh_batch_neighbors_query")
        self.ws_bytes = int(ws.value)
        self.cols_capacity = int(cap.value)

        def grow(buf, n, dtype):
            if buf is None or buf.numel() < n:
                return torch.empty(max(n, 1), dtype=dtype, device=self.device)
            return buf

        self._ws_raw, self.workspace = _workspace(torch, self.ws_bytes, self.device, self._ws_raw)
        if self.kind == "both":
            self.elem_capacity = int(cap2.value)
        if outputs:
            self._rp = grow(self._rp, tot["vert"] + 1, torch.int32)
            self.row_ptr = self._rp[:tot["vert"] + 1]
            self._cols = grow(self._cols, self.cols_capacity, torch.int32)
            self.cols = self._cols
            if self.kind == "both":
                self._erp = grow(self._erp, tot["vert"] + 1, torch.int32)
                self.elem_row_ptr = self._erp[:tot["vert"] + 1]
                self._ecols = grow(self._ecols, self.elem_capacity, torch.int32)
                self.elem_cols = self._ecols
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

    def output_sizes(self):
        """Entries the current batch needs in each output: (row_ptr, cols)
        or, building both, (row_ptr, cols, elem row_ptr, elem cols)."""
        n = self.totals["vert"] + 1
        if self.kind == "both":
            return n, max(self.cols_capacity, 1), n, max(self.elem_capacity, 1)
        return n, max(self.cols_capacity, 1)

    def set_outputs(self, bufs):
        """Write the next launches into the caller's int32 device tensors
        (at least output_sizes() entries each), so that the previous
        launch's results stay valid for whoever still holds them; returns the
        views in use."""
        sizes = self.output_sizes()
        if len(bufs) != len(sizes) or any(b.numel() < n for b, n in zip(bufs, sizes)):
            raise ValueError("output buffers smaller than the batch needs")
        self._rp, self._cols = bufs[0], bufs[1]
        self.row_ptr, self.cols = bufs[0][:sizes[0]], bufs[1]
        if self.kind == "both":
            self._erp, self._ecols = bufs[2], bufs[3]
            self.elem_row_ptr, self.elem_cols = bufs[2][:sizes[2]], bufs[3]
            return self.row_ptr, self.cols, self.elem_row_ptr, self.elem_cols
        return self.row_ptr, self.cols

    def _args(self, conn):
        t = self.totals
        if self.kind == "node":
            a = [_ptr(conn), _ptr(self.segs), self.n_mesh, t["pairs"], t["slots"], t["vert"], t["max_vert"],
                 _ptr(self.row_ptr), _ptr(self.cols), self.cols_capacity]
        elif self.kind == "elem":
            a = [_ptr(conn), _ptr(self.segs), self.n_mesh, t["slots"], t["vert"], _ptr(self.row_ptr),
                 _ptr(self.cols), self.cols_capacity]
        else:
            a = [_ptr(conn), _ptr(self.segs), self.n_mesh, t["pairs"], t["slots"], t["vert"], t["max_vert"],
                 _ptr(self.row_ptr), _ptr(self.cols), self.cols_capacity, _ptr(self.elem_row_ptr),
                 _ptr(self.elem_cols), self.elem_capacity]
        return a + [ctypes.byref(self.options), _ptr(self.workspace), self.ws_bytes]

    def _name(self, prefix="mesh_batch_"):
        return prefix + ("neighbors" if self.kind == "both" else f"{self.kind}_neighbors")

    def launch(self, conn, stream=None):
        import torch

        _check_conn(torch, conn, self.device)
        self._check_conn(conn)
        name = self._name()
        _check(getattr(lib(), name)(*self._args(conn), _stream_handle(stream, self.device)), name)

    def _check_conn(self, conn):
        need = self.totals["ids"]
        if (conn.numel() < need) if self.custom_offsets else (conn.numel() != need):
            raise ValueError(f"conn has {conn.numel()} ids, the segments cover {need}")

    def check(self, stream=None):
        _check(lib().mesh_check(_ptr(self.workspace), _stream_handle(stream, self.device)), "mesh_check")

    def result(self, stream=None):
        self.check(stream)
        nnz = int(self.row_ptr[-1].item())
        if self.kind == "both":
            enz = int(self.elem_row_ptr[-1].item())
            return (self.row_ptr, self.cols[:nnz]), (self.elem_row_ptr, self.elem_cols[:enz])
        return self.row_ptr, self.cols[:nnz]

    def capture(self, conn):
        """A Graph replaying ``launch(conn)`` for the current batch layout
        (totals fixed; conn and segment contents may change between replays
        as long as the totals stay the same)."""
        import torch

        _check_conn(torch, conn, self.device)
        self._check_conn(conn)
        h = _c_p()
        name = self._name("mesh_graph_batch_")
        with _device_guard(self.device):
            st = getattr(lib(), name)(*self._args(conn), ctypes.byref(h))
        _check(st, name)
        # the graph holds the buffers themselves: a later reset() may replace them
        return Graph(h, self.device, keep=(conn, self._ws_raw, self._rp, self._cols, self._erp, self._ecols,
                                           self._segs))

    def mesh_csr(self, m, row_ptr_host=None, relation="node"):
        """(row_ptr, cols) of mesh m alone, as device tensors, after result()
        (relation "elem" for the element CSR of a "both" build)."""
        rp_all, cols_all = ((self.elem_row_ptr, self.elem_cols) if relation == "elem" and self.kind == "both"
                            else (self.row_ptr, self.cols))
        seg = self.seg_host[m]
        v0, nv = int(seg["vert_off"]), int(seg["n_vert"])
        rp = rp_all[v0:v0 + nv + 1]
        if row_ptr_host is not None:
            a, b = int(row_ptr_host[v0]), int(row_ptr_host[v0 + nv])
        else:
            a, b = int(rp[0].item()), int(rp[-1].item())
        return rp - a, cols_all[a:b]


def concat_conn(conns):
    """One int32 array holding the connectivities back to back (row-major)."""
    import numpy as np

    if not conns:
        return np.zeros(0, dtype=np.int32)
    return np.ascontiguousarray(np.concatenate([np.asarray(c, dtype=np.int32).ravel() for c in conns]))
