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
    assert binding.lib().mesh_abi_version() >> 16 == 2
    for st in binding.Status:
        s = binding.status_string(st)
        assert s and s != "unknown status"
    assert binding.status_string(99) == "unknown status"


TYPES = [(0, 3, 3), (1, 6, 4), (2, 12, 8), (3, 4, 4), (4, 9, 6), (5, 8, 5)]


@pytest.mark.parametrize("etype,k,npe", TYPES)
def test_queries(etype, k, npe):
    for ns in (0, 1, 2, 3):
        ws, cap = binding.query_node(1000, etype, 700, {"node_sort": ns})
        assert cap == 2 * k * 1000
        keys = 2 * k * 1000 if ns in (0, 1) else k * 1000 if ns == 2 else npe * 1000
        assert ws >= 2 * 8 * keys  # two key buffers at least
    ws, cap = binding.query_elem(1000, etype, 700)
    assert cap == npe * 1000
    assert ws >= 2 * 8 * cap
    ws, cn, ce = binding.query("both", 1000, etype, 700)
    assert (cn, ce) == (2 * k * 1000, npe * 1000)
    assert binding.query_node(0, etype, 0)[1] == 0


def test_workspace_per_algorithm():
    """Edge-rows sorts one key per element edge (k) instead of two (2k), and
    the element-rows algorithm sorts only the element pairs (npe per
    element): their workspaces are sized for that, so less memory is held."""
    n, v = 1 << 20, 1 << 18
    ws = {ns: binding.query_node(n, 1, v, {"node_sort": ns})[0] for ns in (0, 1, 2, 3)}
    assert ws[2] <= 0.8 * ws[0] and ws[3] <= 0.5 * ws[0]
    both = binding.query("both", n, 1, v, {"node_sort": 3})[0]
    assert both < ws[3]  # the element CSR is the caller's output


def test_query_errors():
    with pytest.raises(binding.MeshError) as e:
        binding.query_node(10, 7, 10)
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
    # the element relation alone needs only its slots below 2^31
    assert binding.query_elem(360_000_000, 0, 3)[1] == 1_080_000_000
    with pytest.raises(binding.MeshError) as e:
        binding.query("both", 360_000_000, 0, 3)
    assert e.value.status == binding.Status.OVERFLOW


@pytest.mark.parametrize("bad", [{"node_sort": 4}, {"node_sort": -2}, {"radix_shape": 7}, {"radix_shape": -5},
                                 {"digit_bits": 9}, {"digit_bits": 0}])
def test_bad_options_refused(bad):
    with pytest.raises(binding.MeshError) as e:
        binding.query_node(100, 0, 60, bad)
    assert e.value.status == binding.Status.INVALID_ARG


def test_default_options():
    o = binding.lib().mesh_default_options()
    assert o.as_dict() == {"node_sort": -1, "radix_shape": -1, "digit_bits": -1}
    # NULL options and all-default options size the same workspace
    w, c = ctypes.c_size_t(0), ctypes.c_int64(0)
    assert binding.lib().mesh_node_neighbors_query(5000, 1, 3000, None, ctypes.byref(w), ctypes.byref(c)) == 0
    assert w.value == binding.query_node(5000, 1, 3000)[0]


def test_options_are_per_call_in_threads():
    """Two threads asking for different algorithms and shapes each get their
    own sizing, call after call: no setting is shared between calls."""
    import threading
    want = {ns: binding.query_node(20000, 1, 5000, {"node_sort": ns, "radix_shape": ns})[0] for ns in (0, 2, 3)}
    assert len(set(want.values())) == 3
    errors = []

    def worker(ns):
        for _ in range(300):
            got = binding.query_node(20000, 1, 5000, {"node_sort": ns, "radix_shape": ns})[0]
            if got != want[ns]:
                errors.append((ns, got))

    th = [threading.Thread(target=worker, args=(ns,)) for ns in want for _ in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors
    assert "mesh_set_node_sort" not in binding.SIGNATURES and not hasattr(binding, "set_node_sort")


@pytest.mark.parametrize("shape", range(7))
def test_radix_launch_shape(shape):
    """Passes over 2^30 keys or more take the default tile (64-bit look-back
    words); below that the requested one.  The batch tile table, histogram
    tiling and staged-id capacity are sized from this same answer."""
    block, items = binding.radix_shapes()[shape]
    assert binding.radix_launch_shape(shape, -1, (1 << 30) - 1) == (block, items, 8)
    assert binding.radix_launch_shape(shape, -1, 1 << 30) == (512, 16, 8)
    assert binding.radix_launch_shape(-1, -1, 1000) == (512, 16, 8)
    with pytest.raises(binding.MeshError):
        binding.radix_launch_shape(7, -1, 10)


def _call(name, conn, n_elem, etype, n_vert, row_ptr, cols, cap, ws, ws_bytes, opts=None):
    return getattr(binding.lib(), name)(ctypes.c_void_p(conn), n_elem, etype, n_vert, ctypes.c_void_p(row_ptr),
                                        ctypes.c_void_p(cols), cap, opts, ctypes.c_void_p(ws), ws_bytes, None)


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
    bad = binding.make_options({"radix_shape": 9})
    assert _call(name, fake, 10, 0, 12, fake, fake, cap, fake, ws_need, ctypes.byref(bad)) == S.INVALID_ARG


def test_mixed_argument_checks():
    lib, S = binding.lib(), binding.Status
    w, c1, c2 = ctypes.c_size_t(0), ctypes.c_int64(0), ctypes.c_int64(0)
    assert lib.mesh_mixed_neighbors_query(10, 40, 100, 30, None, ctypes.byref(w), ctypes.byref(c1),
                                          ctypes.byref(c2)) == 0
    assert (c1.value, c2.value) == (100, 40)
    # the mixed path always derives nodes from elements
    o = binding.make_options({"node_sort": 2})
    assert lib.mesh_mixed_neighbors_query(10, 40, 100, 30, ctypes.byref(o), ctypes.byref(w), ctypes.byref(c1),
                                          ctypes.byref(c2)) == S.INVALID_ARG
    assert lib.mesh_mixed_neighbors_query(10, 2 ** 31, 100, 30, None, ctypes.byref(w), ctypes.byref(c1),
                                          ctypes.byref(c2)) == S.OVERFLOW
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    args = [fake, fake, fake, 10, 40, 100, 30, fake, fake, 100, fake, fake, 40, None, fake, w.value, None]
    a = list(args)
    a[1] = null  # no element offsets
    assert lib.mesh_mixed_neighbors(*a) == S.INVALID_ARG
    a = list(args)
    a[15] = w.value - 1
    assert lib.mesh_mixed_neighbors(*a) == S.WORKSPACE


def test_check_null_workspace_without_a_device():
    """mesh_check(NULL) reads the fixed scratch of mesh_neighbors_noalloc on
    the current device; with no device there is none, and it says so."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    assert binding.lib().mesh_check(None, None) == binding.Status.HIP


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
    w, c, c2 = ctypes.c_size_t(0), ctypes.c_int64(0), ctypes.c_int64(0)
    lib = binding.lib()
    for ns in (0, 1, 2, 3):
        o = binding.make_options({"node_sort": ns})
        assert lib.mesh_batch_node_neighbors_query(3, 1000, 450, 500, 200, ctypes.byref(o), ctypes.byref(w),
                                                   ctypes.byref(c)) == 0
        assert c.value == 1000 and w.value >= 16 * (1000 if ns < 3 else 450)
    assert lib.mesh_batch_elem_neighbors_query(3, 800, 500, None, ctypes.byref(w), ctypes.byref(c)) == 0
    assert c.value == 800
    assert lib.mesh_batch_neighbors_query(3, 1000, 450, 500, 200, None, ctypes.byref(w), ctypes.byref(c),
                                          ctypes.byref(c2)) == 0
    assert (c.value, c2.value) == (1000, 450)
    # max_vert above total_vert is inconsistent
    assert lib.mesh_batch_node_neighbors_query(3, 1000, 450, 100, 200, None, ctypes.byref(w), ctypes.byref(c)) == 1


def test_tuning_table_lookup(tmp_path, monkeypatch):
    import json
    from paper_1604_04689_amd import autotune
    table = {"entries": [
        {"relation": "node", "etype": 0, "bucket": 20, "radix_shape": 2, "node_sort": 1, "digit_bits": 8},
        {"relation": "node", "etype": 0, "bucket": 26, "radix_shape": 0, "node_sort": 3, "digit_bits": 8},
        {"relation": "elem", "etype": 1, "bucket": 24, "radix_shape": 3, "node_sort": -1, "digit_bits": 8},
        {"relation": "batch_both", "etype": -1, "bucket": 28, "radix_shape": 5, "node_sort": 3, "digit_bits": 8}]}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(table))
    monkeypatch.setattr(autotune, "TABLE", str(path))
    monkeypatch.setattr(autotune, "_table_cache", None)
    monkeypatch.delenv("MESHNBR_TUNING", raising=False)
    # 2^20 node pairs of triangles = 174763 elements
    assert autotune.options_for("node", 0, 174763) == {"radix_shape": 2, "digit_bits": 8, "node_sort": 1}
    assert autotune.options_for("node", 0, 8380418)["node_sort"] == 3     # bucket 25 -> nearest 26
    assert autotune.options_for("elem", 1, 5308416) == {"radix_shape": 3, "digit_bits": 8}
    assert autotune.options_for("elem", 0, 1000) is None                    # no entry for the type
    assert autotune.options_for("node", 0, 1000) is None                    # more than two buckets away
    assert autotune.batch_options_for("both", 2 ** 28 + 5, 10) == {"radix_shape": 5, "digit_bits": 8,
                                                                    "node_sort": 3}
    assert autotune.batch_options_for("both", 2 ** 24, 10) is None
    # a build's options come from the table, nothing process-wide changes
    o = binding._resolve("node", 0, 174763, "tuned")
    assert o.as_dict() == {"node_sort": 1, "radix_shape": 2, "digit_bits": 8}
    monkeypatch.setattr(autotune, "_table_cache", None)
    monkeypatch.setenv("MESHNBR_TUNING", "off")
    assert autotune.options_for("node", 0, 174763) is None
    monkeypatch.setattr(autotune, "_table_cache", None)


def test_noalloc_refuses_past_its_scratch_without_a_gpu():
    """mesh_neighbors_noalloc sizes the mesh with the plain query and refuses
    one whose workspace exceeds the fixed scratch before touching the device
    (so this runs without a GPU); bad arguments fail the same way as in
    mesh_neighbors."""
    lib = binding.lib()
    n_elem, n_vert = 3_000_000, 1_600_000
    ws, ncap, ecap = binding.query("both", n_elem, 0, n_vert)
    assert ws > binding.NOALLOC_SCRATCH_BYTES
    st = lib.mesh_neighbors_noalloc(ctypes.c_void_p(16), n_elem, 0, n_vert, ctypes.c_void_p(256), ctypes.c_void_p(256),
                                    ncap, ctypes.c_void_p(256), ctypes.c_void_p(256), ecap, None, None)
    assert st == binding.Status.SCRATCH_LIMIT
    assert lib.mesh_neighbors_noalloc(None, 10, 9, 10, None, None, 0, None, None, 0, None,
                                      None) == binding.Status.UNSUPPORTED_TYPE
    assert lib.mesh_neighbors_noalloc(None, -1, 0, 10, None, None, 0, None, None, 0, None,
                                      None) == binding.Status.INVALID_ARG
