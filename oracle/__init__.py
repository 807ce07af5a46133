"""CPU oracle for one-ring neighbor finding -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (the plain serial definition of
Sec. 1 and Sec. 3.2.2 of the paper, one ordered set per vertex) through
ctypes, and shares no code with the HIP library.

``node_neighbors`` / ``elem_neighbors`` take a host int32 connectivity array
``[n_elem, npe]``, the element type code (0 tri3, 1 tet4, 2 hex8, 3 quad4,
4 wedge6, 5 pyramid5) and the vertex count, and return ``(row_ptr, cols)``
as int32 numpy arrays.  ``mixed_node_neighbors`` / ``mixed_elem_neighbors``
take the ids of all elements back to back and one type code per element.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_NPE = {0: 3, 1: 4, 2: 8, 3: 4, 4: 6, 5: 5}
_EDGES_PER_ELEM = {0: 3, 1: 6, 2: 12, 3: 4, 4: 9, 5: 8}

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it (plain gcc, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
                        _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        for name in ("oracle_node_neighbors", "oracle_elem_neighbors"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int64
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        for name in ("oracle_node_neighbors_mt", "oracle_elem_neighbors_mt"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int64
            fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        for name in ("oracle_mixed_node_neighbors", "oracle_mixed_elem_neighbors"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int64
            fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


_ERRORS = {-1: "invalid argument", -2: "vertex id out of range", -3: "capacity", -4: "out of memory",
           -5: "element offsets do not match its type"}


def _run(fn_name, conn, etype, n_vert, cap_per_elem):
    conn = np.ascontiguousarray(np.asarray(conn, dtype=np.int32))
    npe = _NPE.get(int(etype))
    if npe is None:
        raise OracleError("invalid argument")
    conn = conn.reshape(-1, npe)
    n_elem = conn.shape[0]
    cap = max(1, cap_per_elem * n_elem)
    row_ptr = np.zeros(n_vert + 1, dtype=np.int32)
    cols = np.empty(cap, dtype=np.int32)
    r = getattr(_load(), fn_name)(conn.ctypes.data, n_elem, int(etype), int(n_vert),
                                  row_ptr.ctypes.data, cols.ctypes.data, cap)
    if r < 0:
        raise OracleError(_ERRORS.get(int(r), str(r)))
    return row_ptr, cols[:r].copy()


def node_neighbors(conn, etype: int, n_vert: int):
    """One-ring neighboring nodes of every vertex as (row_ptr, cols)."""
    return _run("oracle_node_neighbors", conn, etype, n_vert, 2 * _EDGES_PER_ELEM.get(int(etype), 0))


def elem_neighbors(conn, etype: int, n_vert: int):
    """One-ring neighboring elements of every vertex as (row_ptr, cols)."""
    return _run("oracle_elem_neighbors", conn, etype, n_vert, _NPE.get(int(etype), 0))


def _run_mixed(fn_name, conn, etypes, n_vert, per_elem):
    conn = np.ascontiguousarray(np.asarray(conn, dtype=np.int32).ravel())
    etypes = np.ascontiguousarray(np.asarray(etypes, dtype=np.int32).ravel())
    npe = np.array([_NPE.get(int(t), 0) for t in etypes], dtype=np.int64)
    elem_off = np.zeros(etypes.shape[0] + 1, dtype=np.int64)
    np.cumsum(npe, out=elem_off[1:])
    if int(elem_off[-1]) != conn.shape[0]:
        raise OracleError("element offsets do not match its type")
    cap = max(1, int(sum(per_elem(int(t)) for t in etypes)))
    row_ptr = np.zeros(n_vert + 1, dtype=np.int32)
    cols = np.empty(cap, dtype=np.int32)
    r = getattr(_load(), fn_name)(conn.ctypes.data, elem_off.ctypes.data, etypes.ctypes.data, etypes.shape[0],
                                  int(n_vert), row_ptr.ctypes.data, cols.ctypes.data, cap)
    if r < 0:
        raise OracleError(_ERRORS.get(int(r), str(r)))
    return row_ptr, cols[:r].copy()


def mixed_node_neighbors(conn, etypes, n_vert: int):
    """Neighboring nodes of a mesh with one type code per element; conn holds
    every element's ids back to back."""
    return _run_mixed("oracle_mixed_node_neighbors", conn, etypes, n_vert, lambda t: 2 * _EDGES_PER_ELEM.get(t, 0))


def mixed_elem_neighbors(conn, etypes, n_vert: int):
    """Neighboring elements of a mesh with one type code per element."""
    return _run_mixed("oracle_mixed_elem_neighbors", conn, etypes, n_vert, lambda t: _NPE.get(t, 0))


def _run_mt(fn_name, conn, etype, n_vert, threads, cap_per_elem):
    conn = np.ascontiguousarray(np.asarray(conn, dtype=np.int32))
    npe = _NPE.get(int(etype))
    if npe is None:
        raise OracleError("invalid argument")
    conn = conn.reshape(-1, npe)
    cap = max(1, cap_per_elem * conn.shape[0])
    row_ptr = np.zeros(n_vert + 1, dtype=np.int32)
    cols = np.empty(cap, dtype=np.int32)
    r = getattr(_load(), fn_name)(conn.ctypes.data, conn.shape[0], int(etype), int(n_vert), int(threads),
                                  row_ptr.ctypes.data, cols.ctypes.data, cap)
    if r < 0:
        raise OracleError(_ERRORS.get(int(r), str(r)))
    return row_ptr, cols[:r].copy()


def node_neighbors_mt(conn, etype: int, n_vert: int, threads: int):
    """node_neighbors on `threads` threads, each owning a vertex range (the
    all-cores CPU baseline); the same result."""
    return _run_mt("oracle_node_neighbors_mt", conn, etype, n_vert, threads, 2 * _EDGES_PER_ELEM.get(int(etype), 0))


def elem_neighbors_mt(conn, etype: int, n_vert: int, threads: int):
    """elem_neighbors on `threads` threads, each owning a vertex range."""
    return _run_mt("oracle_elem_neighbors_mt", conn, etype, n_vert, threads, _NPE.get(int(etype), 0))
