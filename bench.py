#!/usr/bin/env python3
"""Throughput of the one-ring node + element neighbor CSR build on one GPU.

A step is one pass of the whole hot path over one mesh: one mesh_neighbors
call building both relations (the element relation's counting sort of
(vertex, element) pairs by vertex, and the node relation, under the tuned
node algorithm), on one stream, inputs resident in device memory.  Prints ONE
JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload tri2048]

The headline workload is a 2048 x 2048-vertex triangle surface with coin-flip
diagonals (8,380,418 triangles); beside it: the 96^3-cell Kuhn tetrahedral
cube, the 64 x 64 triangle grid (microseconds), the node algorithms compared
on both big meshes, the 512-mesh batch (one batched call vs 512 plain calls
vs 512 graph replays) and the served request stream at offered loads of 0.5,
0.8 and 0.95 of its measured capacity.  Inputs are synthetic (seeded
generators).

The timed steps bracket only the dominant kernel with HIP events (its
duration is the roofline's); the per-kernel table comes from an untimed pass
of as many steps with every launch evented, since each evented launch costs
the stream a few microseconds.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elements/s for node+elem one-ring CSR build (HBM GB/s); batched vs per-mesh"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
EDGES = {0: 3, 1: 6, 2: 12, 3: 4, 4: 9, 5: 8}
NPE = {0: 3, 1: 4, 2: 8, 3: 4, 4: 6, 5: 5}
TYPE_NAME = {0: "tri3", 1: "tet4", 2: "hex8", 3: "quad4", 4: "wedge6", 5: "pyramid5"}
SORT_NAME = {0: "full_key", 1: "vertex_rows", 2: "edge_rows", 3: "elem_rows"}
PROFILES = os.path.join(ROOT, "profiles")

WORKLOADS = {
    "tri2048": ("tri2048_coin: 2048x2048-vertex triangle grid on [0,1]^2, seeded coin-flip diagonal per cell "
                "(8,380,418 tris, 4,194,304 verts), vertex ids permuted, element rows shuffled, int32 conn"),
    "kuhn96": ("kuhn96: 96^3-cell cube, 6 Kuhn tets per cell (5,308,416 tets, 912,673 verts), "
               "vertex ids permuted, element rows shuffled, int32 conn"),
    "tri64": ("tri64_main: 64x64-vertex triangle grid, main diagonals (7,938 tris, 4,096 verts), "
              "ids permuted, rows shuffled"),
}

SERVE_RHO = (0.5, 0.8, 0.95)
# Table 1 of the paper, per row: vertices and triangles of the scanned mesh,
# and its GPU times for the node and the element relation (ms, on a GT640).
# A coin-flip triangle grid of n x n vertices has about the same sizes
# (n^2 vertices, 2 (n-1)^2 triangles); those grids stand in for the meshes.
PAPER_TABLE1 = ((417, "172k", "346k", 50.0, 22.1), (488, "237k", "474k", 66.7, 29.4),
                (573, "327k", "655k", 89.1, 38.3), (661, "437k", "871k", 112.7, 48.5),
                (739, "543k", "1088k", 138.5, 60.6), (940, "882k", "1765k", 221.3, 93.3))
# pair budgets of the bounded-memory build timed on the main workload
CHUNK_BUDGETS = (1 << 20, 1 << 23)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_mesh(name):
    from paper_1604_04689_amd import meshgen as mg
    return {"tri2048": mg.tri2048, "kuhn96": mg.kuhn96, "tri64": mg.tri64}[name]()


def id_bits(n_vert):
    b = 1
    while b < 31 and (1 << b) < n_vert:
        b += 1
    return b


def kernel_bytes(m, nnz_node, nnz_elem, node_sort):
    """Algorithmic HBM bytes per launch of every kernel of a step: what the
    kernel must read and write at least once.  P = directed edge pairs
    (2 x edges per element x F), Q = element pairs (nnz of the element
    relation), U = node nnz, V = vertices, conn = 4 x npe x F bytes.  The
    element sort's last pass reads keys and writes cols and the row starts
    instead of keys, so elem_radix is the mean over its middle passes and that
    last one.  node_erows (rows gathered through the element relation) reads
    the element CSR and conn once and writes each row's distinct values and
    count; node_erows_scan turns the counts into row_ptr and
    node_erows_gather moves the values into cols."""
    f, v, k, npe = m.n_elem, m.n_vert, EDGES[m.etype], NPE[m.etype]
    p_pairs, q_pairs, u = 2 * k * f, nnz_elem, nnz_node
    keys = k * f if node_sort == 2 else p_pairs
    e = u // 2
    conn = 4 * npe * f
    elem_passes = (id_bits(v) + 7) // 8
    csr_out = 4 * q_pairs + 4 * (v + 1)                      # cols and row starts
    later = [16 * q_pairs] * (elem_passes - 2) + [8 * q_pairs + csr_out]
    edge_passes = [16 * e] * (elem_passes - 1) + [8 * e + 4 * e + 4 * (v + 1)]
    return {
        "node_hist": conn,
        "node_radix_first": conn + 8 * keys,
        "node_radix": 16 * keys,
        "node_unique_csr": 8 * keys + 4 * u + 4 * (v + 1),
        "node_row_unique": 8 * keys + 4 * (e if node_sort == 2 else u) + 12 * v,
        "node_row_scan": 8 * v,
        "node_row_gather": 8 * u + 12 * v + 4 * (v + 1),
        "node_long_rows": 0,                                # only rows past the short limit; data-dependent
        "node_edge_transpose": 4 * e + 12 * v + 12 * e,
        "node_edge_hist": 8 * e,
        "node_edge_radix": sum(edge_passes) // len(edge_passes),
        "node_edge_low_fill": 4 * (v + 1),
        "node_edge_merge": 8 * e + 8 * (v + 1) + 4 * u + 4 * (v + 1),
        "node_erows_prep": 4 * (v + 1),                     # element row starts in; tile table (small) out
        "node_erows_long": 0,                               # long rows only; data-dependent
        "node_erows": 4 * (v + 1) + 4 * q_pairs + conn + 4 * v + 4 * u,
        "node_erows_scan": 4 * v + 4 * (v + 1),
        "node_erows_gather": 8 * (v + 1) + 4 * u + 4 * u,
        "hist_sum": 0,
        "elem_hist": conn,
        "elem_radix_first": conn + (8 * q_pairs if elem_passes > 1 else csr_out),
        "elem_radix": sum(later) // len(later) if elem_passes > 1 else 0,
        "elem_row_fill": 4 * (v + 1),
        "fill": 0,
    }


# the translation unit that launches each profiled kernel
KERNEL_UNITS = {"node_erows": "elem_rows.hip"}


def _include_closure(path):
    """path and every file it includes with #include "...", transitively."""
    seen, todo = [], [os.path.normpath(path)]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.append(f)
        with open(f) as fh:
            for line in fh:
                m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
                if m:
                    todo.append(os.path.normpath(os.path.join(os.path.dirname(f), m.group(1))))
    return sorted(seen)


def _code_only(text):
    """Source text without comments and blank space (a comment changes no
    kernel)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(kernel="node_erows"):
    """Hash of the code the kernel is built from (its launching unit and
    every header it includes, comments left out): a traffic record taken on
    other code is stale."""
    h = hashlib.sha256()
    unit = os.path.join(ROOT, "paper_1604_04689_amd", "csrc", KERNEL_UNITS[kernel])
    for f in _include_closure(unit):
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, node_sort):
    """Measured HBM bytes per launch of `kernel` from the committed rocprofv3
    counter summary, or None if absent or taken on other source or with
    another node algorithm."""
    path = os.path.join(PROFILES, f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if kernel not in KERNEL_UNITS or t.get("source_sha") != source_hash(kernel) or t.get("node_sort") != node_sort:
        return None
    return t.get("bytes_per_launch")


def _sync_time(torch, fn, steps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def _snapshot(build):
    outs = [build.row_ptr, build.cols] + ([build.elem_row_ptr, build.elem_cols] if build.kind == "both" else [])
    return [t.clone() for t in outs]


def _same_as(build, snap):
    outs = [build.row_ptr, build.cols] + ([build.elem_row_ptr, build.elem_cols] if build.kind == "both" else [])
    return all(a.shape == b.shape and bool((a == b).all()) for a, b in zip(outs, snap))


def kernel_breakdown(torch, nb, fn, steps):
    """Run fn steps times, untimed, with every kernel launch bracketed by HIP
    events, and return the per-kernel record (timing_read).  Each evented
    launch costs the stream a few microseconds, so the timed steps after it
    bracket only the dominant kernel; this pass gives the rest of the table
    (and leaves the events in the library's pool for the timed steps)."""
    nb.timing_read()
    nb.timing_select(None)
    nb.timing_enable(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    nb.timing_enable(False)
    return nb.timing_read()


def timed_steps(torch, nb, fn, steps, kernel):
    """Seconds per step of fn over `steps` steps between two synchronizations,
    with HIP events around every launch of `kernel` only; returns (seconds,
    that kernel's record (launches, total_ms, min_ms, max_ms) over the same
    steps)."""
    nb.timing_read()
    nb.timing_select([kernel])
    nb.timing_enable(True)
    try:
        sec = _sync_time(torch, fn, steps)
    finally:
        nb.timing_enable(False)
        nb.timing_select(None)
    rec = nb.timing_read().get(kernel)
    if rec is None:
        raise RuntimeError(f"no timed launch of {kernel}")
    return sec, rec


def time_graph(torch, build, conn, stream, steps):
    """Seconds per step of replaying a captured graph of the call; the
    replays must leave exactly the eager outputs."""
    before = _snapshot(build)
    g = build.capture(conn)
    g.launch(stream)
    sec = _sync_time(torch, lambda: g.launch(stream), steps)
    build.check(stream)
    if not _same_as(build, before):
        raise RuntimeError("graph replay differs from the eager result")
    g.destroy()
    return sec


def time_e2e(torch, nb, m, build, steps):
    """Seconds per step including the upload of conn from pinned host memory
    and the download of both CSRs into pinned host memory (context for a
    caller whose mesh lives on the host)."""
    dev = build.device
    host_conn = torch.as_tensor(m.conn).pin_memory()
    conn = torch.empty(host_conn.shape, dtype=torch.int32, device=dev)
    outs = [build.row_ptr, build.cols, build.elem_row_ptr, build.elem_cols]
    host_out = [torch.empty(o.shape, dtype=o.dtype).pin_memory() for o in outs]
    stream = torch.cuda.current_stream(dev)

    def step():
        conn.copy_(host_conn, non_blocking=True)
        build.launch(conn, stream)
        for h, o in zip(host_out, outs):
            h.copy_(o, non_blocking=True)

    step()
    sec = _sync_time(torch, step, steps)
    build.check(stream)
    bytes_moved = host_conn.numel() * 4 + sum(o.numel() * 4 for o in outs)
    return sec, bytes_moved


def run_chunked(torch, nb, m, conn, build, stream, steps, budgets):
    """The bounded-memory build (chunk_keys) of both relations at each pair
    budget: time per step (one wait on the stream per call included),
    workspace against the whole-mesh build's, ranges per call, and byte
    equality with the whole-mesh result."""
    ref = _snapshot(build)
    out = {"whole_mesh_workspace_bytes": build.ws_bytes}
    for cap in budgets:
        b = nb.NeighborBuild("both", m.n_elem, m.etype, m.n_vert, conn.device, options={"chunk_keys": cap})
        b.launch(conn, stream)
        b.check(stream)
        if not _same_as(b, ref):
            raise RuntimeError(f"bounded-memory build (chunk_keys={cap}) differs from the whole-mesh result")
        sec = _sync_time(torch, lambda: b.launch(conn, stream), max(3, steps // 2))
        nb.timing_read()
        nb.timing_enable(True)  # one more call, timed per kernel, to count its ranges
        b.launch(conn, stream)
        torch.cuda.synchronize()
        nb.timing_enable(False)
        ranges = nb.timing_read().get("chunk_compact", (0,))[0]
        out[f"chunk_keys_{cap}"] = {"ms_per_step": sec * 1e3, "elements_per_s": m.n_elem / sec,
                                    "workspace_bytes": b.ws_bytes, "ranges_per_call": ranges}
        log(f"[bench] {m.name} chunk_keys={cap}: {sec * 1e3:.3f} ms/step, {ranges:.0f} ranges, "
            f"workspace {b.ws_bytes / 1e6:.1f} MB (whole mesh {build.ws_bytes / 1e6:.0f} MB)")
        del b
        torch.cuda.empty_cache()
    return out


def run_workload(name, steps, warmup, torch, nb, compare_sorts=True, e2e=True, chunk_budgets=()):
    log(f"[bench] generating {name} ...")
    t = time.time()
    m = make_mesh(name)
    log(f"[bench] {name}: F={m.n_elem} V={m.n_vert} ({time.time() - t:.1f}s)")
    dev = torch.device("cuda:0")
    conn = torch.as_tensor(m.conn).to(dev)
    build = nb.NeighborBuild("both", m.n_elem, m.etype, m.n_vert, dev, options="tuned")
    opts = build.options.as_dict()
    node_sort = opts["node_sort"] if opts["node_sort"] >= 0 else 3
    stream = torch.cuda.current_stream(dev)

    def step():
        build.launch(conn, stream)

    for _ in range(max(warmup, 1)):
        step()
    build.check(stream)
    nnz_node = int(build.row_ptr[-1].item())
    nnz_elem = int(build.elem_row_ptr[-1].item())
    torch.cuda.synchronize()

    # per-kernel table from evented steps (untimed), then the timed steps
    # with events around the dominant kernel only
    kt = kernel_breakdown(torch, nb, step, steps)
    kb = kernel_bytes(m, nnz_node, nnz_elem, node_sort)
    kernels = {}
    model_total = 0
    for k, (launches, total_ms, mn, mx) in sorted(kt.items()):
        per = kb.get(k, 0)
        avg_ms = total_ms / launches
        model_total += per * launches / steps
        kernels[k] = {"launches_per_step": launches / steps, "us_per_step": total_ms / steps * 1e3,
                      "avg_us": avg_ms * 1e3, "bytes_per_launch": per,
                      "GBs": per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 and per else None}
    modeled = {k: v for k, v in kernels.items() if v["bytes_per_launch"]}
    dom = max(modeled, key=lambda k: modeled[k]["us_per_step"])
    sec, dom_rec = timed_steps(torch, nb, step, steps, dom)
    build.check(stream)
    dom_avg_ms = dom_rec[1] / dom_rec[0]

    graph_sec = time_graph(torch, build, conn, stream, steps)
    res = {
        "workload": name,
        "n_elem": m.n_elem, "n_vert": m.n_vert, "etype": TYPE_NAME[m.etype],
        "nnz_node": nnz_node, "nnz_elem": nnz_elem,
        "options": {**opts, "node_sort_name": SORT_NAME[node_sort],
                    "radix_shape": nb.radix_shapes()[opts["radix_shape"]] if opts["radix_shape"] >= 0 else None},
        "radix_passes_elem": sum(kt[k][0] for k in ("elem_radix_first", "elem_radix") if k in kt) // steps,
        "ms_per_step": sec * 1e3,
        "elements_per_s": m.n_elem / sec,
        "graph_ms_per_step": graph_sec * 1e3,
        "graph_elements_per_s": m.n_elem / graph_sec,
        "node_kernel_ms": sum(v[1] for k, v in kt.items() if k.startswith("node_")) / steps,
        "elem_kernel_ms": sum(v[1] for k, v in kt.items() if k.startswith("elem_")) / steps,
        "kernels": kernels,
        "pipeline_model_bytes": model_total,
        "pipeline_model_GBs": model_total / sec / 1e9,
        "pipeline_frac_of_hbm": model_total / sec / 1e9 / HBM_PEAK_GBS,
        "dominant_kernel": {"kernel": dom, "avg_ms": dom_avg_ms, "launches_timed": dom_rec[0],
                            "bytes_per_launch": kernels[dom]["bytes_per_launch"],
                            "GBs": kernels[dom]["bytes_per_launch"] / (dom_avg_ms * 1e-3) / 1e9,
                            "us_per_step": dom_rec[1] / steps * 1e3,
                            "timed": "HIP events around this kernel only, over the timed steps"},
        "kernels_note": "per-kernel figures from the same number of untimed steps with every launch evented",
    }
    log(f"[bench] {name}: {sec * 1e3:.3f} ms/step eager, {graph_sec * 1e3:.3f} ms/step graph replay, "
        f"{m.n_elem / sec / 1e9:.3f} G elem/s ({SORT_NAME[node_sort]}), "
        f"pipeline {res['pipeline_model_GBs']:.0f} GB/s of model bytes")
    for k, v in kernels.items():
        gbs = f"{v['GBs']:7.0f} GB/s" if v["GBs"] else ""
        log(f"[bench]   {k:22s} {v['launches_per_step']:4.1f} x {v['avg_us']:8.1f} us = {v['us_per_step']:8.1f} us/step {gbs}")

    if compare_sorts:
        # every node algorithm on the same mesh, the call building both
        # relations (default tile shape); outputs compared byte for byte
        ref = _snapshot(build)
        by_sort = {}
        for ns in (0, 1, 2, 3):
            b = nb.NeighborBuild("both", m.n_elem, m.etype, m.n_vert, dev, options={"node_sort": ns})
            b.launch(conn, stream)
            b.check(stream)
            if not _same_as(b, ref):
                raise RuntimeError(f"node algorithm {SORT_NAME[ns]} differs from the tuned result")
            s = _sync_time(torch, lambda: b.launch(conn, stream), max(3, steps // 2))
            by_sort[SORT_NAME[ns]] = {"ms_per_step": s * 1e3, "elements_per_s": m.n_elem / s,
                                      "workspace_bytes": b.ws_bytes}
            log(f"[bench] {name} {SORT_NAME[ns]:12s}: {s * 1e3:.3f} ms/step, workspace {b.ws_bytes / 1e6:.0f} MB")
            del b
            torch.cuda.empty_cache()
        res["by_node_sort"] = by_sort
    if chunk_budgets:
        res["chunked"] = run_chunked(torch, nb, m, conn, build, stream, steps, chunk_budgets)
    if e2e:
        s, nbytes = time_e2e(torch, nb, m, build, max(3, steps // 2))
        res["with_transfers"] = {"ms_per_step": s * 1e3, "elements_per_s": m.n_elem / s, "pcie_bytes": nbytes,
                                 "note": "conn uploaded from pinned host memory and both CSRs downloaded to "
                                         "pinned host memory inside each step (context only)"}
        log(f"[bench] {name} with H2D/D2H: {s * 1e3:.3f} ms/step ({nbytes / 1e6:.0f} MB over PCIe)")
    del build, conn
    torch.cuda.empty_cache()
    return m, res


def run_paper_scale(torch, nb, steps=20):
    """Grids sized like the rows of the paper's Table 1: node relation,
    element relation and both, each alone per step (context only: other
    meshes, other hardware)."""
    from paper_1604_04689_amd import meshgen as mg
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rows = []
    for i, (n, pv, pf, p_node, p_elem) in enumerate(PAPER_TABLE1):
        m = mg.tri_grid(n, "coin", mg.BASE_SEED + 100 + i)
        conn = torch.as_tensor(m.conn).to(dev)
        t = {}
        for kind in ("node", "elem", "both"):
            b = nb.NeighborBuild(kind, m.n_elem, m.etype, m.n_vert, dev, options="tuned")
            for _ in range(3):
                b.launch(conn, stream)
            b.check(stream)
            t[kind] = _sync_time(torch, lambda: b.launch(conn, stream), steps) * 1e3
            del b
        rows.append({"table1_row": i + 1, "paper_vertices": pv, "paper_triangles": pf, "grid_side": n,
                     "n_vert": m.n_vert, "n_elem": m.n_elem, "node_ms": t["node"], "elem_ms": t["elem"],
                     "both_ms": t["both"], "paper_gpu_node_ms": p_node, "paper_gpu_elem_ms": p_elem,
                     "node_speedup_vs_paper_gpu": p_node / t["node"], "elem_speedup_vs_paper_gpu": p_elem / t["elem"]})
        log(f"[bench] Table 1 row {i + 1} size ({m.n_elem} tris): node {t['node']:.3f} ms, elem {t['elem']:.3f} ms, "
            f"both {t['both']:.3f} ms (paper GT640: {p_node} / {p_elem} ms)")
        del conn
    torch.cuda.empty_cache()
    return {"note": "coin-flip triangle grids sized like the rows of the paper's Table 1 (its scanned meshes are "
                    "not used); the paper's times are on a GT640 with Thrust (context only)", "rows": rows}


def run_tiny(torch, nb, steps=200):
    """The 64 x 64 grid: microseconds per step, eager and graph replay."""
    m = make_mesh("tri64")
    dev = torch.device("cuda:0")
    conn = torch.as_tensor(m.conn).to(dev)
    b = nb.NeighborBuild("both", m.n_elem, m.etype, m.n_vert, dev, options="tuned")
    stream = torch.cuda.current_stream(dev)
    for _ in range(10):
        b.launch(conn, stream)
    b.check(stream)
    sec = _sync_time(torch, lambda: b.launch(conn, stream), steps)
    gsec = time_graph(torch, b, conn, stream, steps)
    log(f"[bench] tri64: {sec * 1e6:.1f} us/step eager, {gsec * 1e6:.1f} us/step graph replay")
    return {"workload": WORKLOADS["tri64"], "us_per_step": sec * 1e6, "graph_us_per_step": gsec * 1e6,
            "elements_per_s": m.n_elem / sec, "graph_elements_per_s": m.n_elem / gsec,
            "options": b.options.as_dict()}


def run_batched(steps, warmup, torch, nb, per_mesh_steps=2):
    """512 mixed meshes: one batched call (both relations) vs 512 plain
    single-mesh calls vs 512 graph replays, on one stream."""
    from paper_1604_04689_amd import meshgen as mg
    t = time.time()
    meshes = [s.build() for s in mg.batch_specs()]
    log(f"[bench] batch512: {len(meshes)} meshes, F={sum(m.n_elem for m in meshes)} ({time.time() - t:.1f}s)")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    desc = [(m.n_elem, m.etype, m.n_vert) for m in meshes]
    conn = torch.as_tensor(nb.concat_conn([m.conn for m in meshes])).to(dev)
    build = nb.BatchBuild("both", desc, dev, options="tuned")
    total_f = sum(m.n_elem for m in meshes)

    for _ in range(max(warmup, 1)):
        build.launch(conn, stream)
    build.check(stream)
    # per-kernel table from evented steps; the timed steps run without events
    kt = kernel_breakdown(torch, nb, lambda: build.launch(conn, stream), steps)
    batched = _sync_time(torch, lambda: build.launch(conn, stream), steps)
    build.check(stream)
    batched_graph = time_graph(torch, build, conn, stream, steps)
    opts = build.options.as_dict()
    del build
    torch.cuda.empty_cache()

    # the same meshes, one plain call per mesh building both relations
    conns = [torch.as_tensor(m.conn).to(dev) for m in meshes]
    builds = [nb.NeighborBuild("both", m.n_elem, m.etype, m.n_vert, dev, options="tuned") for m in meshes]

    def step_each():
        for c, b in zip(conns, builds):
            b.launch(c, stream)

    step_each()
    per_mesh = _sync_time(torch, step_each, per_mesh_steps)
    for b in builds[:8]:
        b.check(stream)
    graphs = [b.capture(c) for b, c in zip(builds, conns)]

    def replay_each():
        for g in graphs:
            g.launch(stream)

    replay_each()
    per_mesh_graph = _sync_time(torch, replay_each, per_mesh_steps)
    for b in builds[:8]:
        b.check(stream)
    for g in graphs:
        g.destroy()
    del builds, conns, graphs
    torch.cuda.empty_cache()
    res = {"meshes": len(meshes), "n_elem": total_f, "options": opts,
           "batched_ms_per_step": batched * 1e3, "batched_elements_per_s": total_f / batched,
           "batched_graph_ms_per_step": batched_graph * 1e3,
           "per_mesh_ms_per_step": per_mesh * 1e3, "per_mesh_elements_per_s": total_f / per_mesh,
           "per_mesh_graph_ms_per_step": per_mesh_graph * 1e3,
           "batched_over_per_mesh": per_mesh / batched,
           "batched_over_per_mesh_graph": per_mesh_graph / batched,
           "kernel_ms_per_step": {k: v[1] / steps for k, v in sorted(kt.items())},
           "kernels_note": "per-kernel figures from the same number of untimed steps with every launch evented"}
    log(f"[bench] batch512: batched {batched * 1e3:.2f} ms/step ({total_f / batched / 1e9:.2f} G elem/s), "
        f"per-mesh calls {per_mesh * 1e3:.2f} ms/step, per-mesh graph replays {per_mesh_graph * 1e3:.2f} ms/step")
    return meshes, res


def run_serving(meshes, torch, nb, rate_elems=None, n_req=5000, warm=500, slots=4, max_batch=64,
                budget=64 << 30, device_inputs=False):
    """Requests drawn from the batch's meshes, admitted by a device-memory
    budget, continuous batching over `slots` streams.  Inputs start in
    pageable host memory; staging and upload are part of latency.  Arrivals
    are Poisson at `rate_elems` elements/s offered, or all at t = 0
    (saturation: sustained throughput) when rate_elems is None.  With
    device_inputs every request's connectivity is already a device tensor
    (no host staging or upload), which isolates the device side of serving.
    Every retired batch's device error word is checked; any error fails the
    run."""
    import numpy as np
    from paper_1604_04689_amd import meshgen as mg
    from paper_1604_04689_amd import serve
    rng = np.random.default_rng(mg.BASE_SEED + 4)
    pick = rng.integers(0, len(meshes), size=n_req + warm)
    mean_f = float(np.mean([meshes[i].n_elem for i in pick]))
    if rate_elems is None:
        arr = np.zeros(n_req + warm)
    else:
        arr = mg.poisson_arrivals(n_req + warm, rate_elems / mean_f, seed=mg.BASE_SEED + 5)
    ex = serve.GpuExecutor(slots)

    def on_complete(batch, executor):
        executor.check(batch)  # raises MeshError on any device error

    src = {}
    if device_inputs:
        for j in set(int(x) for x in pick):
            src[j] = torch.as_tensor(meshes[j].conn).to("cuda:0")
        torch.cuda.synchronize()
    reqs = [serve.Request(i, float(t), src.get(int(j), meshes[j].conn), meshes[j].etype, meshes[j].n_vert)
            for i, (j, t) in enumerate(zip(pick, arr))]
    ex.warm(reqs, max_batch)  # device buffers sized up front: no allocation while serving
    with serve.frozen_gc():  # no full collector pass inside the serving loop
        srv = serve.Server(ex, serve.RealClock(), n_slots=slots, budget_bytes=budget, max_batch=max_batch,
                           on_complete=on_complete)
        t0 = time.perf_counter()
        done = srv.run(reqs)
        wall = time.perf_counter() - t0
    measured = sorted(done, key=lambda r: r.rid)[warm:]  # the first `warm` arrivals are warm-up
    summ = serve.latency_summary(measured)
    summ.update({"offered_elements_per_s": rate_elems, "arrivals": "poisson" if rate_elems else "all at t=0",
                 "slots": slots, "max_batch": max_batch, "budget_bytes": budget, "batches": srv.batches,
                 "mean_batch": float(np.mean(srv.batch_sizes)), "peak_reserved_bytes": srv.peak_in_use,
                 "wall_s": wall, "warmup_requests": warm, "errors_checked": True,
                 "inputs": "device tensors" if device_inputs else "pageable host arrays (staged and uploaded)",
                 "input_GBs": sum(4 * meshes[pick[r.rid]].conn.size for r in measured) / summ["span_s"] / 1e9})
    what = f"offered {rate_elems / 1e9:.2f} G elem/s" if rate_elems else "saturation"
    if device_inputs:
        what += ", device inputs"
    log(f"[bench] serve ({what}): {summ['requests']} requests: p50 {summ['p50_ms']:.2f} ms, "
        f"p99 {summ['p99_ms']:.2f} ms, {summ['elements_per_s'] / 1e9:.2f} G elem/s sustained, "
        f"{srv.batches} batches")
    return summ


def _host_cpu():
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return os.cpu_count(), model


def cpu_baseline(m):
    """The oracle on the headline mesh: single thread (the oracle as it
    stands), and the all-cores variant (threads own vertex ranges)."""
    import oracle
    t0 = time.perf_counter()
    oracle.node_neighbors(m.conn, m.etype, m.n_vert)
    t1 = time.perf_counter()
    oracle.elem_neighbors(m.conn, m.etype, m.n_vert)
    t2 = time.perf_counter()
    nproc, model = _host_cpu()
    out = {"value": m.n_elem / (t2 - t0), "unit": "elements/s", "cores": 1, "kind": "oracle",
           "sample": f"the full {m.n_elem}-element mesh, node then element relation, one pass, single thread "
                     f"(node {t1 - t0:.2f} s + elem {t2 - t1:.2f} s)",
           "host": {"nproc": nproc, "cpu_model": model}}
    threads = max(1, min(nproc or 1, 64))
    t0 = time.perf_counter()
    oracle.node_neighbors_mt(m.conn, m.etype, m.n_vert, threads)
    oracle.elem_neighbors_mt(m.conn, m.etype, m.n_vert, threads)
    t1 = time.perf_counter()
    out["all_cores"] = {"value": m.n_elem / (t1 - t0), "unit": "elements/s", "cores": threads,
                        "sample": "the same mesh, each thread owning a vertex range and scanning every element"}
    return out


def copy_calibration(torch, gib=2):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {gib} GiB")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="tri2048", choices=sorted(WORKLOADS))
    ap.add_argument("--also", default="kuhn96", help="comma list of extra workloads reported beside ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-mesh batch and the serving stream")
    ap.add_argument("--no-compare", action="store_true", help="skip the node-algorithm comparison")
    ap.add_argument("--no-paper-scale", action="store_true", help="skip the grids sized like the paper's Table 1")
    ap.add_argument("--serve-requests", type=int, default=5000)
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (for counter scaling under rocprofv3)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the neighbor build has no multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU (torch.cuda.is_available() is False)", file=sys.stderr)
        sys.exit(1)
    import paper_1604_04689_amd as nb
    nb.lib()

    if args.copy_calibration:
        copy_calibration(torch)

    m, main_res = run_workload(args.workload, args.steps, args.warmup, torch, nb, compare_sorts=not args.no_compare,
                               chunk_budgets=CHUNK_BUDGETS if not args.no_compare else ())
    others = {}
    for w in [x for x in args.also.split(",") if x and x != args.workload]:
        _, others[w] = run_workload(w, args.steps, args.warmup, torch, nb, compare_sorts=not args.no_compare)
    others["tri64"] = run_tiny(torch, nb)
    if not args.no_paper_scale:
        others["paper_scale"] = run_paper_scale(torch, nb)

    if not args.no_batch:
        meshes, others["batch512"] = run_batched(max(3, args.steps // 4), 1, torch, nb)
        sat = run_serving(meshes, torch, nb, rate_elems=None, n_req=args.serve_requests, warm=args.serve_warmup)
        others["serve_saturation"] = sat
        others["serve_saturation_device_inputs"] = run_serving(meshes, torch, nb, rate_elems=None,
                                                               n_req=args.serve_requests, warm=args.serve_warmup,
                                                               device_inputs=True)
        capacity = sat["elements_per_s"]
        others["serve"] = {f"rho_{rho}": run_serving(meshes, torch, nb, rate_elems=rho * capacity,
                                                     n_req=args.serve_requests, warm=args.serve_warmup)
                           for rho in SERVE_RHO}
        others["serve"]["capacity_elements_per_s"] = capacity
        others["serve"]["capacity_note"] = ("capacity = the sustained rate of the served path at saturation "
                                            "(uploads from host memory included); offered load = rho x capacity")
        del meshes

    dom = main_res["dominant_kernel"]
    traffic = load_traffic(dom["kernel"], args.workload, main_res["options"]["node_sort"])
    roofline = {"bound": "hbm", "achieved": dom["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dom["GBs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom["kernel"],
                "algorithmic_bytes_per_launch": dom["bytes_per_launch"], "avg_launch_ms": dom["avg_ms"],
                "pipeline_frac": main_res["pipeline_frac_of_hbm"]}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        cpu = cpu_baseline(m)
        log(f"[bench] oracle: {cpu['value']:.3e} elements/s ({cpu['sample']}); all cores: "
            f"{cpu['all_cores']['value']:.3e} elements/s on {cpu['all_cores']['cores']} threads")

    out = {
        "metric": METRIC,
        "value": main_res["elements_per_s"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n_elem": m.n_elem, "n_vert": m.n_vert,
                   "etype": TYPE_NAME[m.etype], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": main_res,
        "also": others,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
