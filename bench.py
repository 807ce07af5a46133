#!/usr/bin/env python3
"""Throughput of the one-ring node + element neighbor CSR build on one GPU.

A step is one pass of the whole hot path over one mesh: the node pipeline
(pair emission, LSD radix sort, unique/CSR) and the element pipeline
(counting sort by vertex, row sort), both on one stream, inputs resident in
device memory.  Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload tri2048]

The headline workload is a 2048 x 2048-vertex triangle surface with coin-flip
diagonals (8,380,418 triangles); the 96^3-cell Kuhn tetrahedral cube is
measured beside it.  Inputs are synthetic (seeded generators).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elements/s for node+elem one-ring CSR build (HBM GB/s); batched vs per-mesh"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
EDGES = {0: 3, 1: 6, 2: 12}
NPE = {0: 3, 1: 4, 2: 8}
TYPE_NAME = {0: "tri3", 1: "tet4", 2: "hex8"}
PROFILES = os.path.join(ROOT, "profiles")

WORKLOADS = {
    "tri2048": ("tri2048_coin: 2048x2048-vertex triangle grid on [0,1]^2, seeded coin-flip diagonal per cell "
                "(8,380,418 tris, 4,194,304 verts), vertex ids permuted, element rows shuffled, int32 conn"),
    "kuhn96": ("kuhn96: 96^3-cell cube, 6 Kuhn tets per cell (5,308,416 tets, 912,673 verts), "
               "vertex ids permuted, element rows shuffled, int32 conn"),
    "tri64": ("tri64_main: 64x64-vertex triangle grid, main diagonals (7,938 tris, 4,096 verts), "
              "ids permuted, rows shuffled"),
}


SERVE_OFFERED = 0.6e9  # elements/s offered to the serving stream (Poisson arrivals)


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
    """Algorithmic HBM bytes per launch of every kernel of the two pipelines:
    what the kernel must read and write at least once.  P = directed edge
    pairs (2 x edges per element x F), Q = element pairs (nnz of the element
    relation), U = node nnz, V = vertices, conn = 4 x npe x F bytes.  The node
    sort passes move K keys: P, or with the edge-rows algorithm the k x F
    canonical edge keys; E = U / 2 unique edges.  The element sort's last
    pass reads keys and writes cols and the row starts instead of keys, so
    elem_radix is the mean over its middle passes and that last one."""
    f, v, k, npe = m.n_elem, m.n_vert, EDGES[m.etype], NPE[m.etype]
    p_pairs, q_pairs, u = 2 * k * f, nnz_elem, nnz_node
    keys = k * f if node_sort == 2 else p_pairs
    e = u // 2
    conn = 4 * npe * f
    id_bits = max(1, (v - 1).bit_length())
    elem_passes = (id_bits + 7) // 8
    csr_out = 4 * q_pairs + 4 * (v + 1)                      # cols and row starts
    later = [16 * q_pairs] * (elem_passes - 2) + [8 * q_pairs + csr_out]
    # edge passes sort the E transposed edges by their higher vertex (id_bits);
    # the last one writes the lower neighbours and their group starts
    edge_passes = [16 * e] * (elem_passes - 1) + [8 * e + 4 * e + 4 * (v + 1)]
    return {
        "node_hist": conn,                                  # read conn
        "node_radix_first": conn + 8 * keys,                # read conn, write keys
        "node_radix": 16 * keys,                            # read + write keys
        "node_unique_csr": 8 * keys + 4 * u + 4 * (v + 1),
        "node_row_unique": 8 * keys + 4 * (e if node_sort == 2 else u) + 12 * v,  # keys in; row values + deg/src out
        "node_row_scan": 8 * v,
        "node_row_gather": 8 * u + 12 * v + 4 * (v + 1),
        "node_long_rows": 0,                                # only rows past the short limit; data-dependent
        "node_edge_transpose": 4 * e + 12 * v + 12 * e,     # row values, up_ptr/deg/src in; keys + ids out
        "node_edge_hist": 8 * e,
        "node_edge_radix": sum(edge_passes) // len(edge_passes),
        "node_edge_low_fill": 4 * (v + 1),
        "node_edge_merge": 8 * e + 8 * (v + 1) + 4 * u + 4 * (v + 1),
        "elem_hist": conn,
        "elem_radix_first": conn + (8 * q_pairs if elem_passes > 1 else csr_out),
        "elem_radix": sum(later) // len(later) if elem_passes > 1 else 0,
        "elem_row_fill": 4 * (v + 1),                       # block minima, then the fill: each reads row_ptr
        "fill": 0,
    }


def radix_source_hash():
    h = hashlib.sha256()
    for f in ("radix.hpp", "common.hpp", "launch.hpp"):
        with open(os.path.join(ROOT, "paper_1604_04689_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload, node_sort):
    """HBM bytes per node_radix launch from the committed rocprofv3 counter
    summary, or None if absent, taken on different kernel source, or with a
    different node algorithm (which changes the keys per launch)."""
    path = os.path.join(PROFILES, f"node_radix_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha") != radix_source_hash() or t.get("node_sort") != node_sort:
        return None
    return t.get("bytes_per_launch")


def time_graph_replays(torch, graphs, builds, stream, steps):
    """Seconds per step of replaying the captured graphs; checks that the
    replays leave exactly the eager outputs in place."""
    before = [(b.row_ptr.clone(), b.cols.clone()) for b in builds]
    for g in graphs:
        g.launch(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for g in graphs:
            g.launch(stream)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    for b, (rp, cols) in zip(builds, before):
        b.check(stream)
        nnz = int(rp[-1].item())
        if not (torch.equal(b.row_ptr, rp) and torch.equal(b.cols[:nnz], cols[:nnz])):
            raise RuntimeError("graph replay differs from the eager result")
    for g in graphs:
        g.destroy()
    return sec


def time_two_streams(torch, node, elem, conn, stream, steps):
    """Seconds per step with the two relations on two streams (they are
    independent, so their radix passes overlap); outputs checked against the
    sequential ones."""
    side = torch.cuda.Stream(conn.device)
    before = [(b.row_ptr.clone(), b.cols.clone()) for b in (node, elem)]

    def step():
        ev = torch.cuda.Event()
        ev.record(stream)
        side.wait_event(ev)
        node.launch(conn, stream, tuned=True)
        elem.launch(conn, side, tuned=True)
        back = torch.cuda.Event()
        back.record(side)
        stream.wait_event(back)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    for b, (rp, cols) in zip((node, elem), before):
        b.check(stream)
        nnz = int(rp[-1].item())
        if not (torch.equal(b.row_ptr, rp) and torch.equal(b.cols[:nnz], cols[:nnz])):
            raise RuntimeError("two-stream step differs from the sequential result")
    return sec


def run_workload(name, steps, warmup, torch, nb):
    log(f"[bench] generating {name} ...")
    t = time.time()
    m = make_mesh(name)
    log(f"[bench] {name}: F={m.n_elem} V={m.n_vert} ({time.time() - t:.1f}s)")
    dev = torch.device("cuda:0")
    conn = torch.as_tensor(m.conn).to(dev)
    node = nb.NeighborBuild("node", m.n_elem, m.etype, m.n_vert, dev)
    elem = nb.NeighborBuild("elem", m.n_elem, m.etype, m.n_vert, dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        node.launch(conn, stream, tuned=True)
        elem.launch(conn, stream, tuned=True)

    for _ in range(max(warmup, 1)):
        step()
    node.check(stream)
    elem.check(stream)
    nnz_node = int(node.row_ptr[-1].item())
    nnz_elem = int(elem.row_ptr[-1].item())
    torch.cuda.synchronize()

    nb.timing_read()  # clear
    nb.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nb.timing_enable(False)
    kt = nb.timing_read()
    node.check(stream)
    elem.check(stream)

    sec = (t1 - t0) / steps
    graph_sec = time_graph_replays(torch, [node.capture(conn, tuned=True), elem.capture(conn, tuned=True)],
                                   [node, elem], stream, steps)
    two_sec = time_two_streams(torch, node, elem, conn, stream, steps)
    from paper_1604_04689_amd import autotune
    tuned = {kind: autotune.lookup(kind, m.etype, m.n_elem) for kind in ("node", "elem")}
    node_sort = tuned["node"]["mode"] if tuned["node"] else 0
    tuned = {kind: (None if e is None else {"shape": nb.radix_shapes()[e["shape"]], "node_sort": e["mode"]})
             for kind, e in tuned.items()}
    kb = kernel_bytes(m, nnz_node, nnz_elem, node_sort)
    kernels = {}
    model_total = 0
    for k, (launches, total_ms, mn, mx) in sorted(kt.items()):
        per = kb.get(k, 0)
        avg_ms = total_ms / launches
        model_total += per * launches / steps
        kernels[k] = {"launches_per_step": launches / steps, "us_per_step": total_ms / steps * 1e3,
                      "avg_us": avg_ms * 1e3, "bytes_per_launch": per,
                      "GBs": per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else None}
    node_p = sum(kt[k][0] for k in ("node_radix_first", "node_radix") if k in kt) // steps
    elem_p = sum(kt[k][0] for k in ("elem_radix_first", "elem_radix") if k in kt) // steps
    node_ms = sum(v[1] for k, v in kt.items() if k.startswith("node_")) / steps
    elem_ms = sum(v[1] for k, v in kt.items() if k.startswith("elem_")) / steps
    res = {
        "workload": name,
        "n_elem": m.n_elem, "n_vert": m.n_vert, "etype": TYPE_NAME[m.etype],
        "nnz_node": nnz_node, "nnz_elem": nnz_elem, "radix_passes": {"node": node_p, "elem": elem_p}, "tuned": tuned,
        "ms_per_step": sec * 1e3,
        "elements_per_s": m.n_elem / sec,
        "graph_ms_per_step": graph_sec * 1e3,
        "two_streams_ms_per_step": two_sec * 1e3,
        "two_streams_elements_per_s": m.n_elem / two_sec,
        "node_kernel_ms": node_ms, "elem_kernel_ms": elem_ms,
        "kernels": kernels,
        "pipeline_model_bytes": model_total,
        "pipeline_model_GBs": model_total / sec / 1e9,
        "pipeline_frac_of_hbm": model_total / sec / 1e9 / HBM_PEAK_GBS,
        "radix_pass": {"kernel": "node_radix", "avg_ms": kernels["node_radix"]["avg_us"] * 1e-3,
                       "bytes_per_launch": kb["node_radix"], "GBs": kernels["node_radix"]["GBs"]},
    }
    log(f"[bench] {name}: {sec * 1e3:.3f} ms/step eager, {graph_sec * 1e3:.3f} ms/step graph replay, "
        f"{two_sec * 1e3:.3f} ms/step on two streams, "
        f"{m.n_elem / sec / 1e9:.3f} G elem/s, "
        f"pipeline {res['pipeline_model_GBs']:.0f} GB/s of model bytes")
    for k, v in kernels.items():
        gbs = f"{v['GBs']:7.0f} GB/s" if v["GBs"] else ""
        log(f"[bench]   {k:18s} {v['launches_per_step']:4.1f} x {v['avg_us']:8.1f} us = {v['us_per_step']:8.1f} us/step {gbs}")
    del node, elem, conn
    torch.cuda.empty_cache()
    return m, res


def run_batched(steps, warmup, torch, nb, per_mesh_steps=2):
    """512 mixed meshes: one batched launch sequence per relation vs 512
    plain single-mesh calls per relation, on one stream."""
    from paper_1604_04689_amd import meshgen as mg
    t = time.time()
    meshes = [s.build() for s in mg.batch_specs()]
    log(f"[bench] batch512: {len(meshes)} meshes, F={sum(m.n_elem for m in meshes)} ({time.time() - t:.1f}s)")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    desc = [(m.n_elem, m.etype, m.n_vert) for m in meshes]
    conn = torch.as_tensor(nb.concat_conn([m.conn for m in meshes])).to(dev)
    node = nb.BatchBuild("node", desc, dev)
    elem = nb.BatchBuild("elem", desc, dev)
    total_f = sum(m.n_elem for m in meshes)

    def step():
        node.launch(conn, stream, tuned=True)
        elem.launch(conn, stream, tuned=True)

    for _ in range(max(warmup, 1)):
        step()
    node.check(stream)
    elem.check(stream)
    nb.timing_read()
    nb.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nb.timing_enable(False)
    kt = nb.timing_read()
    node.check(stream)
    elem.check(stream)
    batched = (t1 - t0) / steps
    batched_graph = time_graph_replays(torch, [node.capture(conn, tuned=True), elem.capture(conn, tuned=True)],
                                       [node, elem], stream, steps)
    del node, elem

    # the same meshes, one plain call per mesh and relation
    conns = [torch.as_tensor(m.conn).to(dev) for m in meshes]
    builds = [(nb.NeighborBuild("node", m.n_elem, m.etype, m.n_vert, dev),
               nb.NeighborBuild("elem", m.n_elem, m.etype, m.n_vert, dev)) for m in meshes]

    def step_each():
        for c, (bn, be) in zip(conns, builds):
            bn.launch(c, stream, tuned=True)
            be.launch(c, stream, tuned=True)

    step_each()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(per_mesh_steps):
        step_each()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for bn, be in builds[:8]:
        bn.check(stream)
        be.check(stream)
    per_mesh = (t1 - t0) / per_mesh_steps
    del builds, conns
    torch.cuda.empty_cache()
    res = {"meshes": len(meshes), "n_elem": total_f,
           "batched_ms_per_step": batched * 1e3, "batched_elements_per_s": total_f / batched,
           "batched_graph_ms_per_step": batched_graph * 1e3,
           "per_mesh_ms_per_step": per_mesh * 1e3, "per_mesh_elements_per_s": total_f / per_mesh,
           "batched_over_per_mesh": per_mesh / batched,
           "kernel_ms_per_step": {k: v[1] / steps for k, v in sorted(kt.items())}}
    log(f"[bench] batch512: batched {batched * 1e3:.2f} ms/step ({total_f / batched / 1e9:.2f} G elem/s), "
        f"per-mesh calls {per_mesh * 1e3:.2f} ms/step ({total_f / per_mesh / 1e9:.2f} G elem/s)")
    return meshes, res


def run_serving(meshes, torch, nb, rate_elems=None, n_req=600, warm=60, slots=4, max_batch=32,
                budget=64 << 30):
    """Requests drawn from the batch's meshes, admitted by a device-memory
    budget for their buffers, continuous batching over `slots` streams.
    Inputs start in pageable host memory; staging and upload are part of
    latency.  Arrivals are Poisson at `rate_elems` elements/s offered, or all
    at t = 0 (saturation: sustained throughput) when rate_elems is None."""
    import numpy as np
    from paper_1604_04689_amd import meshgen as mg
    from paper_1604_04689_amd import serve
    rng = np.random.default_rng(mg.BASE_SEED + 4)
    pick = rng.integers(0, len(meshes), size=n_req + warm)
    mean_f = float(np.mean([meshes[i].n_elem for i in pick]))
    if rate_elems is None:
        arr = np.zeros(n_req)
    else:
        arr = mg.poisson_arrivals(n_req, rate_elems / mean_f, seed=mg.BASE_SEED + 5)
    ex = serve.GpuExecutor(slots)
    # warm-up stream on the same executor (pinned staging blocks, device buffers), not measured
    warm_reqs = [serve.Request(i, 0.0, meshes[j].conn, meshes[j].etype, meshes[j].n_vert)
                 for i, j in enumerate(pick[n_req:])]
    serve.Server(ex, serve.RealClock(), n_slots=slots, budget_bytes=budget, max_batch=max_batch).run(warm_reqs)
    reqs = [serve.Request(i, float(t), meshes[j].conn, meshes[j].etype, meshes[j].n_vert)
            for i, (j, t) in enumerate(zip(pick[:n_req], arr))]
    srv = serve.Server(ex, serve.RealClock(), n_slots=slots, budget_bytes=budget, max_batch=max_batch)
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    summ = serve.latency_summary(done)
    summ.update({"offered_elements_per_s": rate_elems, "arrivals": "poisson" if rate_elems else "all at t=0",
                 "slots": slots, "max_batch": max_batch, "budget_bytes": budget, "batches": srv.batches,
                 "mean_batch": float(np.mean(srv.batch_sizes)), "peak_reserved_bytes": srv.peak_in_use,
                 "wall_s": wall, "warmup_requests": warm})
    what = f"offered {rate_elems / 1e9:.2f} G elem/s" if rate_elems else "saturation"
    log(f"[bench] serve ({what}): {summ['requests']} requests: p50 {summ['p50_ms']:.2f} ms, "
        f"p99 {summ['p99_ms']:.2f} ms, {summ['elements_per_s'] / 1e9:.2f} G elem/s sustained, "
        f"{srv.batches} batches")
    return summ


def cpu_baseline(m):
    import oracle
    t0 = time.perf_counter()
    oracle.node_neighbors(m.conn, m.etype, m.n_vert)
    t1 = time.perf_counter()
    oracle.elem_neighbors(m.conn, m.etype, m.n_vert)
    t2 = time.perf_counter()
    return {"value": m.n_elem / (t2 - t0), "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"the full {m.n_elem}-element mesh, node then element relation, one pass, single thread "
                      f"(node {t1 - t0:.2f} s + elem {t2 - t1:.2f} s)"}


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
    ap.add_argument("--serve-requests", type=int, default=600)
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

    m, main_res = run_workload(args.workload, args.steps, args.warmup, torch, nb)
    others = {}
    for w in [x for x in args.also.split(",") if x and x != args.workload]:
        _, others[w] = run_workload(w, args.steps, args.warmup, torch, nb)

    if not args.no_batch:
        meshes, others["batch512"] = run_batched(max(3, args.steps // 4), 1, torch, nb)
        others["serve"] = run_serving(meshes, torch, nb, rate_elems=SERVE_OFFERED, n_req=args.serve_requests)
        others["serve_saturation"] = run_serving(meshes, torch, nb, rate_elems=None, n_req=args.serve_requests)
        del meshes

    traffic = load_traffic(args.workload, (main_res["tuned"]["node"] or {}).get("node_sort", 0))
    rp = main_res["radix_pass"]
    roofline = {"bound": "hbm", "achieved": rp["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": rp["GBs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": rp["kernel"],
                "algorithmic_bytes_per_launch": rp["bytes_per_launch"], "avg_launch_ms": rp["avg_ms"]}

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        cpu = cpu_baseline(m)
        log(f"[bench] oracle: {cpu['value']:.3e} elements/s ({cpu['sample']})")

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
        "dtype": "u64",
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
