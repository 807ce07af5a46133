"""Autotuner for the library's speed-only choices.

Every choice it makes changes speed only, never results: the radix tile
shape (threads per block x keys per thread, which also sets the number of
tiles in flight per CU) and, for the node relation, the algorithm (LSD sort
of the full key; sort by the vertex bits plus per-row deduplication; or each
edge once by its lower vertex, deduplicated per row, then transposed).
For each workload it times every combination on the GPU, checks that all of
them produce byte-identical CSR output, and records the fastest per
(relation, element type, size bucket) in ``tuning.json`` next to this file.
``NeighborBuild.launch(..., tuned=True)`` applies the table before the
launch; without ``tuned`` the process-wide settings are left as they are
(set ``MESHNBR_TUNING=off`` to ignore the table).

    python -m paper_1604_04689_amd.autotune [--quick]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import time

from . import binding as _b

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")


def size_bucket(n_keys: int) -> int:
    """log2 bucket of the number of keys a relation sorts."""
    return max(0, int(math.log2(max(n_keys, 1))))


def keys_of(kind, n_elem, etype):
    npe = _b.NODES_PER_ELEM[etype]
    return 2 * _b.EDGES_PER_ELEM[etype] * n_elem if kind == "node" else npe * n_elem


_table_cache = None


def load_table():
    global _table_cache
    if _table_cache is None:
        if os.environ.get("MESHNBR_TUNING", "").lower() == "off" or not os.path.exists(TABLE):
            _table_cache = {}
        else:
            with open(TABLE) as fh:
                data = json.load(fh)
            _table_cache = {(e["relation"], e["etype"], e["bucket"]): e for e in data.get("entries", [])}
    return _table_cache


def _nearest(relation, etype, n_keys):
    table = load_table()
    if not table:
        return None
    b = size_bucket(n_keys)
    best = None
    for (rel, et, bk), e in table.items():
        if rel == relation and et == etype and (best is None or abs(bk - b) < abs(best["bucket"] - b)):
            best = e
    return best


def lookup(kind, etype, n_elem):
    """The tuned entry for a single-mesh call, or the nearest bucket of the
    same relation and type, or None."""
    return _nearest(kind, etype, keys_of(kind, n_elem, etype))


def lookup_batch(kind, n_keys):
    """The tuned entry for a batch of n_keys pairs (node) or slots (element)."""
    return _nearest("batch_" + kind, -1, n_keys)


def _set(kind, e):
    if e is None:
        _b.set_radix_shape(-1)
        if kind == "node":
            _b.set_node_sort(_b.NODE_SORT_FULL_KEY)
        return
    _b.set_radix_shape(e["shape"])
    if kind == "node":
        _b.set_node_sort(e["mode"])


def apply(kind, etype, n_elem):
    _set(kind, lookup(kind, etype, n_elem))


def apply_batch(kind, n_keys):
    _set(kind, lookup_batch(kind, n_keys))


def _digest(row_ptr, cols):
    h = hashlib.sha256()
    h.update(row_ptr.cpu().numpy().tobytes())
    h.update(cols.cpu().numpy().tobytes())
    return h.hexdigest()


def time_config(torch, kind, mesh, conn, shape, mode, steps):
    _b.set_radix_shape(shape)
    if kind == "node":
        _b.set_node_sort(mode)
    build = _b.NeighborBuild(kind, mesh.n_elem, mesh.etype, mesh.n_vert, conn.device)
    build.launch(conn)
    rp, cols = build.result()
    digest = _digest(rp, cols)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        build.launch(conn)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    build.check()
    del build
    return ms, digest


def time_batch_config(torch, kind, desc, conn, shape, mode, steps):
    _b.set_radix_shape(shape)
    if kind == "node":
        _b.set_node_sort(mode)
    build = _b.BatchBuild(kind, desc, conn.device)
    build.launch(conn)
    rp, cols = build.result()
    digest = _digest(rp, cols)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        build.launch(conn)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    build.check()
    del build
    return ms, digest


def tune_batches(torch, batches, steps=3, log=print):
    entries = []
    for name, meshes in batches:
        desc = [(m.n_elem, m.etype, m.n_vert) for m in meshes]
        conn = torch.as_tensor(_b.concat_conn([m.conn for m in meshes])).to("cuda:0")
        seg, tot = _b.segment_table(desc)
        for kind in ("node", "elem"):
            modes = (0, 1, 2) if kind == "node" else (0,)
            results = []
            for mode in modes:
                for shape in range(len(_b.radix_shapes())):
                    ms, dg = time_batch_config(torch, kind, desc, conn, shape, mode, steps)
                    results.append((ms, shape, mode, dg))
                    log(f"[tune] {name} batch {kind} shape {_b.radix_shapes()[shape]} mode {mode}: {ms:.3f} ms")
            if len({r[3] for r in results}) != 1:
                raise RuntimeError(f"configurations disagree on batch {name} {kind}: outputs differ")
            ms, shape, mode, _ = min(results)
            n_keys = tot["pairs"] if kind == "node" else tot["slots"]
            entries.append({"relation": "batch_" + kind, "etype": -1, "bucket": size_bucket(n_keys),
                            "shape": shape, "mode": mode, "ms": ms, "workload": name,
                            "candidates": {f"shape{s}_mode{md}": round(t, 4) for t, s, md, _ in results}})
        del conn
        torch.cuda.empty_cache()
    return entries


def tune(meshes, steps=5, log=print, batches=()):
    import torch

    entries = []
    dev = torch.device("cuda:0")
    for m in meshes:
        conn = torch.as_tensor(m.conn).to(dev)
        for kind in ("node", "elem"):
            modes = (0, 1, 2) if kind == "node" else (0,)
            results = []
            for mode in modes:
                for shape in range(len(_b.radix_shapes())):
                    ms, dg = time_config(torch, kind, m, conn, shape, mode, steps)
                    results.append((ms, shape, mode, dg))
                    log(f"[tune] {m.name} {kind} shape {_b.radix_shapes()[shape]} mode {mode}: {ms:.3f} ms")
            if len({r[3] for r in results}) != 1:
                raise RuntimeError(f"configurations disagree on {m.name} {kind}: outputs differ")
            ms, shape, mode, _ = min(results)
            entries.append({"relation": kind, "etype": m.etype, "bucket": size_bucket(keys_of(kind, m.n_elem, m.etype)),
                            "shape": shape, "mode": mode, "ms": ms, "workload": m.name,
                            "candidates": {f"shape{s}_mode{md}": round(t, 4) for t, s, md, _ in results}})
        del conn
        torch.cuda.empty_cache()
    entries += tune_batches(torch, batches, log=log)
    _b.set_radix_shape(-1)
    _b.set_node_sort(_b.NODE_SORT_FULL_KEY)
    props = torch.cuda.get_device_properties(0)
    return {"device": getattr(props, "gcnArchName", props.name), "shapes": _b.radix_shapes(), "entries": entries}


def main():
    from . import meshgen as mg

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--quick", action="store_true", help="small meshes only")
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    if args.quick:
        meshes = [mg.tri_grid(256, "coin", 1), mg.kuhn_tet_grid(16, 2), mg.hex_grid(16, 3)]
        batches = [("batch64", [s.build() for s in mg.batch_specs(64, seed=7)])]
    else:
        meshes = [mg.tri_grid(256, "coin", 1), mg.tri_grid(1024, "coin", 2), mg.tri2048(),
                  mg.kuhn_tet_grid(24, 3), mg.kuhn_tet_grid(48, 4), mg.kuhn96(),
                  mg.hex_grid(24, 5), mg.hex_grid(64, 6)]
        batches = [("batch64", [s.build() for s in mg.batch_specs(64, seed=7)]),
                   ("batch512", [s.build() for s in mg.batch_specs()])]
    table = tune(meshes, batches=batches)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(f"wrote {args.out} with {len(table['entries'])} entries", flush=True)


if __name__ == "__main__":
    main()
