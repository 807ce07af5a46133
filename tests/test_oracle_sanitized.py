"""The oracle built with the address and undefined-behaviour sanitizers (gcc,
host code only) on the golden cases and random meshes of every type, mixed
meshes, degenerate elements and refused inputs: no sanitizer report, and the
same bytes as the plain build.  CPU only."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests import pins

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")
DRIVER_C = os.path.join(HERE, "oracle_driver.c")


def _records():
    recs = []
    for c in pins.read_golden():
        recs.append((0, c["etype"], c["n_vert"], c["conn"], None))
    for c in pins.read_golden("mixed_cases.txt"):
        recs.append((1, 0, c["n_vert"], c["conn"], c["etypes"]))
    for et in range(6):
        for seed, (ne, nv) in enumerate([(0, 5), (1, 1), (40, 9), (700, 300)]):
            m = mg.random_mesh(ne, nv, et, seed=seed + 10 * et)
            recs.append((0, et, nv, m.conn.ravel(), None))
            recs.append((2, et, nv, m.conn.ravel(), None))
    for seed in range(4):
        m = mg.random_mixed(200 * seed, 50 + seed, seed)
        recs.append((1, 0, m.n_vert, m.conn, m.etypes))
    recs.append((1, 0, 6, mg.hybrid_grid(2, 3).conn, mg.hybrid_grid(2, 3).etypes))
    recs.append((0, 0, 3, np.array([0, 1, 3]), None))       # id out of range: refused
    recs.append((1, 0, 4, np.array([0, 1, 2, 3]), np.array([0])))  # offsets disagree with the type: refused
    return recs


def _write(path, recs):
    with open(path, "wb") as fh:
        for kind, et, nv, ids, types in recs:
            ids = np.ascontiguousarray(ids, dtype=np.int32).ravel()
            n_elem = len(types) if kind == 1 else (ids.size // pins.NPE[et])
            fh.write(struct.pack("<iiiqq", kind, et, nv, n_elem, ids.size))
            fh.write(ids.tobytes())
            if kind == 1:
                fh.write(np.ascontiguousarray(types, dtype=np.int32).tobytes())


def _run(exe, path):
    r = subprocess.run([exe, path], capture_output=True, timeout=600,
                       env={**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                            "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert r.returncode == 0, r.stderr.decode()[-3000:]
    assert b"runtime error" not in r.stderr and b"AddressSanitizer" not in r.stderr, r.stderr.decode()[-3000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_sanitizers(tmp_path):
    recs = _records()
    data = tmp_path / "in.bin"
    _write(data, recs)
    outs = {}
    for name, flags in (("plain", ["-O2"]), ("sanitized", ["-O1", "-g", "-fsanitize=address,undefined",
                                                            "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"])):
        exe = str(tmp_path / name)
        subprocess.run(["gcc", "-std=c99", "-Wall", *flags, ORACLE_C, DRIVER_C, "-pthread", "-o", exe], check=True)
        outs[name] = _run(exe, str(data))
    assert outs["plain"] == outs["sanitized"]
    # and the outputs are the oracle's answers: spot-check the parse of the
    # first record against the golden values
    r = struct.unpack_from("<q", outs["plain"], 0)[0]
    c = pins.read_golden()[0]
    assert r == c["node_cols"].shape[0]
