"""Host-side logic of bench.py that needs no GPU: the multi-GPU refusal, the
staleness key of the committed traffic records, and the byte model's inputs."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_code_only_drops_comments_and_spacing():
    a = "int a;  // note\n/* block\n comment */ int b;\n"
    b = "int a;\nint b; /* other words */"
    assert bench._code_only(a) == bench._code_only(b) == "int a; int b;"
    assert bench._code_only("int a;") != bench._code_only("int c;")


def test_source_hash_covers_the_kernels_includes():
    files = [os.path.basename(f) for f in bench._include_closure(
        os.path.join(ROOT, "paper_1604_04689_amd", "csrc", bench.KERNEL_UNITS["node_erows"]))]
    assert {"elem_rows.hip", "erows.hpp", "common.hpp", "mesh_neighbors.h"} <= set(files)
    assert len(bench.source_hash()) == 16


def test_traffic_records_are_reported_only_for_their_code():
    """The committed node_erows records carry the hash of the code they were
    taken on; bench.py reports one only while that hash matches the present
    code, and only for the node algorithm it was taken with."""
    for w in ("tri2048", "kuhn96"):
        path = os.path.join(bench.PROFILES, f"node_erows_{w}_traffic.json")
        rec = json.load(open(path))
        fresh = rec["source_sha"] == bench.source_hash()
        want = rec["bytes_per_launch"] if fresh else None
        assert bench.load_traffic("node_erows", w, rec["node_sort"]) == want
        assert bench.load_traffic("node_erows", w, 0) is None
        assert rec["bytes_per_launch"] > rec["algorithmic_bytes"] > 0
    assert bench.load_traffic("elem_radix", "tri2048", 3) is None
