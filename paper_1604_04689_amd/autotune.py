"""Autotuner for the library's speed-only choices.

Every choice it makes changes speed only, never results: the node algorithm
(LSD sort of the full key; sort by the vertex bits plus per-row
deduplication; each edge once by its lower vertex, deduplicated per row, then
transposed; or rows gathered through the element relation), the radix tile
shape (threads per block x keys per thread, which also sets the waves per
block and, through the LDS a tile needs, the blocks and so waves per CU) and
the radix digit width (8 or 11 bits, for the element sort).  For each workload it times every combination on the
GPU, checks that all of them produce byte-identical CSR output, and records
the fastest per (relation, element type, size bucket) in ``tuning.json`` next
to this file.

The table is read once and never written by a running program; a build asks
for its options with ``options_for`` / ``batch_options_for`` and passes them
to each call (``mesh_options``), so nothing process-wide changes.  A size
more than two buckets away from every entry of its relation and type gets the
library defaults.  Set ``MESHNBR_TUNING=off`` to ignore the table.

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
MAX_BUCKET_GAP = 2
# the tile shapes the tuner times (the others never won a sweep over all of
# them on MI355X; they stay selectable through mesh_options)
TUNED_SHAPES = (0, 2, 4, 5)
# 11-bit digits apply to the element sort (the element relation, and the node
# relation under the element-rows algorithm); the wide pass has one tile shape
WIDE_SHAPE = 0


def size_bucket(n_keys: int) -> int:
    """log2 bucket of the number of keys a relation sorts."""
    return max(0, int(math.log2(max(n_keys, 1))))


def keys_of(kind, n_elem, etype):
    """Pairs (node relation, both relations) or slots (element relation)."""
    if kind == "elem":
        return _b.NODES_PER_ELEM[etype] * n_elem
    return 2 * _b.EDGES_PER_ELEM[etype] * n_elem


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
    b = size_bucket(n_keys)
    best = None
    for (rel, et, bk), e in load_table().items():
        if rel == relation and et == etype and abs(bk - b) <= MAX_BUCKET_GAP and (
                best is None or abs(bk - b) < abs(best["bucket"] - b)):
            best = e
    return best


def _as_options(e, kind):
    if e is None:
        return None
    o = {"radix_shape": e["radix_shape"], "digit_bits": e.get("digit_bits", -1)}
    if kind != "elem":
        o["node_sort"] = e["node_sort"]
    return o


def options_for(kind, etype, n_elem):
    """mesh_options (as a dict) for a single-mesh call of relation kind
    ("node", "elem" or "both"), or None for the library defaults."""
    return _as_options(_nearest(kind, etype, keys_of(kind, n_elem, etype)), kind)


def batch_options_for(kind, pairs, slots):
    """mesh_options (as a dict) for a batch of `pairs` directed pairs and
    `slots` node slots, or None."""
    return _as_options(_nearest("batch_" + kind, -1, slots if kind == "elem" else pairs), kind)


def _digest(out):
    h = hashlib.sha256()
    if isinstance(out[0], tuple):
        for rp, cols in out:
            h.update(rp.cpu().numpy().tobytes())
            h.update(cols.cpu().numpy().tobytes())
    else:
        h.update(out[0].cpu().numpy().tobytes())
        h.update(out[1].cpu().numpy().tobytes())
    return h.hexdigest()


def _time(torch, build, conn, steps):
    build.launch(conn)
    digest = _digest(build.result())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        build.launch(conn)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    build.check()
    return ms, digest


def candidates(kind, batch=False):
    """Every (node algorithm, tile shape, digit width) timed for a relation:
    8-bit digits under every tuned shape, 11-bit digits (the element sort
    only; batches sort with 8-bit digits) under the wide pass's shape."""
    modes = (0, 1, 2, 3) if kind != "elem" else (-1,)
    out = []
    for m in modes:
        out += [{"node_sort": m, "radix_shape": s, "digit_bits": 8} for s in TUNED_SHAPES]
        if not batch and (kind != "node" or m == 3):
            out.append({"node_sort": m, "radix_shape": WIDE_SHAPE, "digit_bits": 11})
    return out


def _entry(relation, etype, n_keys, results, workload):
    if len({r[2] for r in results}) != 1:
        raise RuntimeError(f"configurations disagree on {workload} {relation}: outputs differ")
    ms, opts, _ = min(results, key=lambda r: r[0])
    return {"relation": relation, "etype": etype, "bucket": size_bucket(n_keys), **opts, "ms": ms,
            "workload": workload,
            "candidates": {f"ns{o['node_sort']}_shape{o['radix_shape']}_d{o['digit_bits']}": round(t, 4)
                           for t, o, _ in results}}


def tune(meshes, steps=5, log=print, batches=()):
    import torch

    entries = []
    dev = torch.device("cuda:0")
    for m in meshes:
        conn = torch.as_tensor(m.conn).to(dev)
        for kind in ("node", "elem", "both"):
            results = []
            for o in candidates(kind):
                b = _b.NeighborBuild(kind, m.n_elem, m.etype, m.n_vert, dev, options=o)
                ms, dg = _time(torch, b, conn, steps)
                del b
                results.append((ms, o, dg))
                log(f"[tune] {m.name} {kind} {o}: {ms:.3f} ms")
            entries.append(_entry(kind, m.etype, keys_of(kind, m.n_elem, m.etype), results, m.name))
        del conn
        torch.cuda.empty_cache()
    for name, meshes_b in batches:
        desc = [(x.n_elem, x.etype, x.n_vert) for x in meshes_b]
        conn = torch.as_tensor(_b.concat_conn([x.conn for x in meshes_b])).to(dev)
        _, tot = _b.segment_table(desc)
        for kind in ("node", "elem", "both"):
            results = []
            for o in candidates(kind, batch=True):
                b = _b.BatchBuild(kind, desc, dev, options=o)
                ms, dg = _time(torch, b, conn, max(2, steps // 2))
                del b
                results.append((ms, o, dg))
                log(f"[tune] {name} batch {kind} {o}: {ms:.3f} ms")
            entries.append(_entry("batch_" + kind, -1, tot["slots"] if kind == "elem" else tot["pairs"], results,
                                  name))
        del conn
        torch.cuda.empty_cache()
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
        meshes = [mg.tri64(), mg.tri_grid(256, "coin", 1), mg.tri_grid(512, "coin", 7), mg.tri_grid(1024, "coin", 2),
                  mg.tri2048(), mg.kuhn_tet_grid(24, 3), mg.kuhn_tet_grid(34, 8), mg.kuhn_tet_grid(48, 4), mg.kuhn96(),
                  mg.hex_grid(24, 5), mg.hex_grid(40, 9), mg.hex_grid(64, 6)]
        batches = [("batch64", [s.build() for s in mg.batch_specs(64, seed=7)]),
                   ("batch512", [s.build() for s in mg.batch_specs()])]
    table = tune(meshes, batches=batches)
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(f"wrote {args.out} with {len(table['entries'])} entries", flush=True)


if __name__ == "__main__":
    main()
