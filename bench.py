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


def model_bytes(m, nnz_node, nnz_elem):
    """Algorithmic HBM bytes of the pipeline as run (bytes each kernel must
    move at least once): node = conn + key write + p radix passes (read and
    write) + unique read + cols + row_ptr; elem = two conn reads + cols
    scatter + row-sort read/write + counts/scan/row_ptr."""
    f, v, k, npe = m.n_elem, m.n_vert, EDGES[m.etype], NPE[m.etype]
    p_pairs = 2 * k * f
    passes = -(-2 * id_bits(v) // 8)
    node = 4 * npe * f + 8 * p_pairs + passes * 16 * p_pairs + 8 * p_pairs + 4 * nnz_node + 4 * (v + 1)
    elem = 2 * 4 * npe * f + 4 * nnz_elem + 8 * nnz_elem + 12 * (v + 1)
    return node, elem, passes


def radix_source_hash():
    h = hashlib.sha256()
    for f in ("node_path.hip", "common.hpp", "launch.hpp"):
        with open(os.path.join(ROOT, "paper_1604_04689_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload):
    """HBM bytes per radix_pass launch from the committed rocprofv3 counter
    summary, or None if absent or taken on different kernel source."""
    path = os.path.join(PROFILES, f"radix_pass_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha") != radix_source_hash():
        return None
    return t.get("bytes_per_launch")


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
        node.launch(conn, stream)
        elem.launch(conn, stream)

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
    n_pairs = 2 * EDGES[m.etype] * m.n_elem
    node_b, elem_b, passes = model_bytes(m, nnz_node, nnz_elem)
    launches, total_ms, _, _ = kt["radix_pass"]
    radix_ms = total_ms / launches
    radix_bytes = 16 * n_pairs
    node_kernels = ("node_emit", "radix_pass", "unique_csr")
    node_ms = sum(v[1] for k, v in kt.items() if k in node_kernels) / steps
    all_ms = sum(v[1] for v in kt.values()) / steps
    res = {
        "workload": name,
        "n_elem": m.n_elem, "n_vert": m.n_vert, "etype": TYPE_NAME[m.etype],
        "nnz_node": nnz_node, "nnz_elem": nnz_elem, "radix_passes": passes,
        "ms_per_step": sec * 1e3,
        "elements_per_s": m.n_elem / sec,
        "kernel_ms_per_step": {k: v[1] / steps for k, v in sorted(kt.items())},
        "kernel_launches_per_step": {k: v[0] / steps for k, v in sorted(kt.items())},
        "node_kernel_ms": node_ms, "elem_kernel_ms": all_ms - node_ms,
        "model_bytes": {"node": node_b, "elem": elem_b},
        "pipeline_model_GBs": (node_b + elem_b) / sec / 1e9,
        "pipeline_frac_of_hbm": (node_b + elem_b) / sec / 1e9 / HBM_PEAK_GBS,
        "radix_pass": {"avg_ms": radix_ms, "bytes_per_launch": radix_bytes,
                       "GBs": radix_bytes / (radix_ms * 1e-3) / 1e9},
    }
    log(f"[bench] {name}: {sec * 1e3:.3f} ms/step, {m.n_elem / sec / 1e9:.3f} G elem/s, "
        f"radix {radix_ms * 1e3:.1f} us = {res['radix_pass']['GBs']:.0f} GB/s")
    for k, v in sorted(kt.items()):
        log(f"[bench]   {k:14s} {v[0] / steps:5.1f} launches  {v[1] / steps * 1e3:9.1f} us/step")
    del node, elem, conn
    torch.cuda.empty_cache()
    return m, res


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

    traffic = load_traffic(args.workload)
    rp = main_res["radix_pass"]
    roofline = {"bound": "hbm", "achieved": rp["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": rp["GBs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": "radix_pass",
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
