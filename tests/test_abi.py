"""The C-ABI library loads, exports every symbol its header declares, and its
host-only paths (queries, status strings, argument checks that return before
anything is launched) behave as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

from paper_1604_04689_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(mesh_[a-z_]+)\s*\(", text, flags=re.M)
    return names


def test_header_parsed():
    names = _declared_functions()
    assert "mesh_node_neighbors" in names and "mesh_elem_neighbors" in names and "mesh_check" in names


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert set(_declared_functions()) <= set(binding.SIGNATURES)


def test_version_and_status_strings():
    assert binding.lib().mesh_abi_version() >> 16 == 1
    for st in binding.Status:
        s = binding.status_string(st)
        assert s and s != "unknown status"
    assert binding.status_string(99) == "unknown status"


@pytest.mark.parametrize("etype,k,npe", [(0, 3, 3), (1, 6, 4), (2, 12, 8)])
def test_queries(etype, k, npe):
    ws, cap = binding.query_node(1000, etype, 700)
    assert cap == 2 * k * 1000
    assert ws >= 2 * 8 * cap  # two key buffers at least
    ws, cap = binding.query_elem(1000, etype, 700)
    assert cap == npe * 1000
    assert ws >= 4 * 700  # per-vertex cursors
    assert binding.query_node(0, etype, 0)[1] == 0


def test_query_errors():
    with pytest.raises(binding.MeshError) as e:
        binding.query_node(10, 5, 10)
    assert e.value.status == binding.Status.UNSUPPORTED_TYPE
    with pytest.raises(binding.MeshError) as e:
        binding.query_elem(-1, 0, 10)
    assert e.value.status == binding.Status.INVALID_ARG
    with pytest.raises(binding.MeshError) as e:
        binding.query_node(2 ** 31 // 6 + 1, 0, 10)
    assert e.value.status == binding.Status.OVERFLOW
    with pytest.raises(binding.MeshError) as e:
        binding.query_elem(2 ** 31 // 8 + 1, 2, 10)
    assert e.value.status == binding.Status.OVERFLOW


def _call(name, conn, n_elem, etype, n_vert, row_ptr, cols, cap, ws, ws_bytes):
    return getattr(binding.lib(), name)(ctypes.c_void_p(conn), n_elem, etype, n_vert, ctypes.c_void_p(row_ptr),
                                        ctypes.c_void_p(cols), cap, ctypes.c_void_p(ws), ws_bytes, None)


@pytest.mark.parametrize("name", ["mesh_node_neighbors", "mesh_elem_neighbors"])
def test_argument_checks_return_before_launch(name):
    # fake (never dereferenced) addresses: every call below must be refused on the host
    fake = 0x100000
    kind = name.split("_")[1]
    ws_need, cap = getattr(binding, f"query_{kind}")(10, 0, 12)
    S = binding.Status
    assert _call(name, fake, 10, 7, 12, fake, fake, cap, fake, ws_need) == S.UNSUPPORTED_TYPE
    assert _call(name, fake, -1, 0, 12, fake, fake, cap, fake, ws_need) == S.INVALID_ARG
    assert _call(name, fake, 10, 0, -3, fake, fake, cap, fake, ws_need) == S.INVALID_ARG
    assert _call(name, 0, 10, 0, 12, fake, fake, cap, fake, ws_need) == S.INVALID_ARG      # null conn
    assert _call(name, fake, 10, 0, 12, 0, fake, cap, fake, ws_need) == S.INVALID_ARG      # null row_ptr
    assert _call(name, fake, 10, 0, 12, fake, 0, cap, fake, ws_need) == S.INVALID_ARG      # null cols
    assert _call(name, fake, 10, 0, 12, fake, fake, -1, fake, ws_need) == S.INVALID_ARG    # negative cap
    assert _call(name, fake, 10, 0, 12, fake, fake, cap, 0, ws_need) == S.INVALID_ARG      # null workspace
    assert _call(name, fake, 10, 0, 12, fake, fake, cap, fake, ws_need - 1) == S.WORKSPACE  # too small
    assert _call(name, fake, 10, 0, 12, fake, fake, cap, fake + 4, ws_need) == S.WORKSPACE  # misaligned


def test_check_null_workspace():
    assert binding.lib().mesh_check(None, None) == binding.Status.INVALID_ARG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="missing"):
        binding.lib()


def test_segment_table_offsets():
    seg, tot = binding.segment_table([(10, 0, 12), (0, 1, 5), (3, 2, 20), (7, 1, 9)])
    assert seg.dtype.itemsize == 48
    assert seg["conn_off"].tolist() == [0, 30, 30, 54]
    assert seg["pair_off"].tolist() == [0, 60, 60, 132]
    assert seg["slot_off"].tolist() == [0, 30, 30, 54]
    assert seg["vert_off"].tolist() == [0, 12, 17, 37]
    assert tot == {"pairs": 132 + 84, "slots": 54 + 28, "vert": 46, "ids": 82, "max_vert": 20}


def test_batch_queries():
    ws, cap = 0, 0
    import ctypes
    w, c = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert binding.lib().mesh_batch_node_neighbors_query(3, 1000, 500, 200, ctypes.byref(w), ctypes.byref(c)) == 0
    assert c.value == 1000 and w.value >= 16 * 1000
    assert binding.lib().mesh_batch_elem_neighbors_query(3, 800, 500, ctypes.byref(w), ctypes.byref(c)) == 0
    assert c.value == 800
    # max_vert above total_vert is inconsistent
    assert binding.lib().mesh_batch_node_neighbors_query(3, 1000, 100, 200, ctypes.byref(w), ctypes.byref(c)) == 1


def test_tuning_table_lookup(tmp_path, monkeypatch):
    import json
    from paper_1604_04689_amd import autotune
    table = {"entries": [
        {"relation": "node", "etype": 0, "bucket": 20, "shape": 2, "mode": 1},
        {"relation": "node", "etype": 0, "bucket": 26, "shape": 0, "mode": 0},
        {"relation": "elem", "etype": 1, "bucket": 24, "shape": 3, "mode": 0}]}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(table))
    monkeypatch.setattr(autotune, "TABLE", str(path))
    monkeypatch.setattr(autotune, "_table_cache", None)
    monkeypatch.delenv("MESHNBR_TUNING", raising=False)
    # 2^20 node pairs of triangles = 174763 elements
    assert autotune.lookup("node", 0, 174763)["shape"] == 2
    assert autotune.lookup("node", 0, 8380418)["mode"] == 0      # bucket 25 -> nearest 26
    assert autotune.lookup("elem", 1, 5308416)["shape"] == 3
    assert autotune.lookup("elem", 0, 1000) is None               # no entry for the type
    autotune.apply("node", 0, 174763)
    assert binding.get_radix_shape() == 2 and binding.get_node_sort() == 1
    autotune.apply("elem", 0, 10)
    assert binding.get_radix_shape() == 0
    binding.set_node_sort(0)
    monkeypatch.setattr(autotune, "_table_cache", None)
    monkeypatch.setenv("MESHNBR_TUNING", "off")
    assert autotune.lookup("node", 0, 174763) is None
    monkeypatch.setattr(autotune, "_table_cache", None)
