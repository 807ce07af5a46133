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


def test_timing_selection_arguments():
    """The timing selection is host state only: lists of launch names are
    taken, too long a list or too many names are refused and leave the
    selection as it was."""
    lib = binding.lib()
    ok, bad = binding.Status.OK, binding.Status.INVALID_ARG
    assert lib.mesh_timing_select(None) == ok
    assert lib.mesh_timing_select(b"") == ok
    assert lib.mesh_timing_select(b"node_erows") == ok
    assert lib.mesh_timing_select(b"node_erows,elem_radix,,fill") == ok
    assert lib.mesh_timing_select(b"x" * 1025) == bad
    assert lib.mesh_timing_select(",".join(f"k{i}" for i in range(33)).encode()) == bad
    assert lib.mesh_timing_select(",".join(f"k{i}" for i in range(32)).encode()) == ok
    binding.timing_select(["node_erows", "fill"])
    binding.timing_select(None)
    with pytest.raises(binding.MeshError):
        binding.timing_select(["y" * 1100])


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
    assert o.as_dict() == {"node_sort": -1, "radix_shape": -1, "digit_bits": -1, "chunk_keys": -1}
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
    assert o.as_dict() == {"node_sort": 1, "radix_shape": 2, "digit_bits": 8, "chunk_keys": -1}
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


# ---- bounded-memory build (mesh_options.chunk_keys) --------------------------

@pytest.mark.parametrize("bad", [{"chunk_keys": 4095}, {"chunk_keys": 1}, {"chunk_keys": -2},
                                 {"chunk_keys": 4096, "node_sort": 0}, {"chunk_keys": 4096, "node_sort": 2},
                                 {"chunk_keys": 4096, "digit_bits": 11}])
def test_chunk_options_refused(bad):
    """A budget below 4096 pairs, a node algorithm other than ELEM_ROWS for a
    call that builds the node relation, or 11-bit digits."""
    for kind in ("node", "both"):
        with pytest.raises(binding.MeshError) as e:
            binding.query(kind, 1000, 0, 600, bad)
        assert e.value.status == binding.Status.INVALID_ARG


def test_chunk_options_accepted():
    # the element relation alone ignores the node algorithm
    assert binding.query("elem", 1000, 0, 600, {"chunk_keys": 4096, "node_sort": 0})[1] == 3000
    # -1 and 0 mean the whole mesh: the same workspace as no option
    for k in (-1, 0):
        assert binding.query("node", 5000, 1, 3000, {"chunk_keys": k}) == binding.query("node", 5000, 1, 3000)
    # capacities do not depend on the budget
    assert binding.query("both", 5000, 1, 3000, {"chunk_keys": 8192})[1:] == binding.query("both", 5000, 1, 3000)[1:]


def test_chunk_budget_covers_one_bin():
    """Ranges are cut at bins of the top 11 vertex bits: a budget below one
    bin's vertices (2^20 of them for 31-bit ids) is refused."""
    with pytest.raises(binding.MeshError) as e:
        binding.query("node", 1000, 0, 2 ** 31 - 1, {"chunk_keys": (1 << 20) - 1})
    assert e.value.status == binding.Status.INVALID_ARG
    binding.query("node", 1000, 0, 2 ** 31 - 1, {"chunk_keys": 1 << 20})
    binding.query("node", 1000, 0, 1 << 15, {"chunk_keys": 4096})   # bins of 16 vertices


@pytest.mark.parametrize("etype", [0, 1, 2])
def test_chunk_workspace_is_bounded(etype):
    """The whole-mesh build takes 17 to 50 bytes per connectivity slot; the
    bounded build takes O(chunk_keys) plus one 8-byte look-back word per 24576
    slots (the compaction's tiles)."""
    npe = binding.NODES_PER_ELEM[etype]
    n_elem, n_vert, cap = 4_000_000, 1_500_000, 1 << 20
    for kind in ("node", "elem", "both"):
        whole = binding.query(kind, n_elem, etype, n_vert)[0]
        a = binding.query(kind, n_elem, etype, n_vert, {"chunk_keys": cap})[0]
        b = binding.query(kind, 2 * n_elem, etype, n_vert, {"chunk_keys": cap})[0]
        assert whole >= 17 * npe * n_elem
        assert a < whole / 4
        assert abs((b - a) - npe * n_elem * 8 / 24576) < 512    # 8 bytes per 24576 added slots
        assert a < 80 * cap + (4 << 20)                          # O(cap) otherwise


def test_chunk_refused_for_batches_mixed_and_graphs():
    lib = binding.lib()
    o = binding.make_options({"chunk_keys": 8192})
    w, c, c2 = ctypes.c_size_t(0), ctypes.c_int64(0), ctypes.c_int64(0)
    assert lib.mesh_batch_node_neighbors_query(3, 1000, 450, 500, 200, ctypes.byref(o), ctypes.byref(w),
                                               ctypes.byref(c)) == binding.Status.INVALID_ARG
    assert lib.mesh_batch_elem_neighbors_query(3, 800, 500, ctypes.byref(o), ctypes.byref(w),
                                               ctypes.byref(c)) == binding.Status.INVALID_ARG
    assert lib.mesh_mixed_neighbors_query(100, 400, 800, 300, ctypes.byref(o), ctypes.byref(w), ctypes.byref(c),
                                          ctypes.byref(c2)) == binding.Status.INVALID_ARG
    # a capture cannot hold the histogram read-back: refused before capturing
    # (so without a device), and the handle cleared
    g = ctypes.c_void_p(1)
    st = lib.mesh_graph_node_neighbors(ctypes.c_void_p(256), 10, 0, 10, ctypes.c_void_p(256), ctypes.c_void_p(256),
                                       60, ctypes.byref(o), ctypes.c_void_p(256), 1 << 20, ctypes.byref(g))
    assert st == binding.Status.INVALID_ARG and not g.value


def test_chunk_lets_noalloc_take_larger_meshes():
    """The no-allocation entry sizes with the plain query: a mesh past its
    scratch as a whole fits it under a pair budget."""
    n_elem, n_vert = 3_000_000, 1_600_000
    assert binding.query("both", n_elem, 0, n_vert)[0] > binding.NOALLOC_SCRATCH_BYTES
    assert binding.query("both", n_elem, 0, n_vert, {"chunk_keys": 1 << 20})[0] < binding.NOALLOC_SCRATCH_BYTES
