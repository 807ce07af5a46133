"""Parity of the element sort with 11-bit digit passes (mesh_options.digit_bits
= 11) against the CPU oracle, through the C ABI.  Both relations are exact
integer work with one canonical answer: bit-exact, tolerance 0.

The wide pass is taken when it needs fewer passes than 8-bit digits over the
vertex bits: 9..11 bits (one pass, which reads the connectivity and writes
the CSR), 17..22 bits (two passes), 25..31 bits (three)."""
import numpy as np
import pytest

from paper_1604_04689_amd import meshgen as mg
from tests.test_gpu_parity import assert_same, gpu_csr

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

WIDE = {"digit_bits": 11}


@pytest.mark.parametrize("etype", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("n_vert", [300, 1500, 70_000, 3_000_000])
def test_wide_passes_random(oracle_mod, etype, n_vert):
    """Random connectivity (degenerate and duplicate elements, unused
    vertices), several 8192-key tiles with a ragged tail."""
    n_elem = 25_013 if etype != 2 else 9_001
    m = mg.random_mesh(n_elem, n_vert, etype, seed=700 + etype + n_vert % 97)
    print(f"[wide] etype={etype} n_elem={n_elem} n_vert={n_vert}", flush=True)
    we = oracle_mod.elem_neighbors(m.conn, etype, n_vert)
    wn = oracle_mod.node_neighbors(m.conn, etype, n_vert)
    assert_same(gpu_csr("elem", m.conn, etype, n_vert, options=WIDE), we, "wide elem")
    gn, ge = gpu_csr("both", m.conn, etype, n_vert, options=WIDE)
    assert_same(ge, we, "wide both/elem")
    assert_same(gn, wn, "wide both/node")


@pytest.mark.parametrize("n_vert", [1 << 11, (1 << 22), (1 << 25) + 3])
def test_wide_digit_boundaries(oracle_mod, n_vert):
    """Vertex counts at the edges of the bit ranges: 11 bits (one wide pass of
    exactly 11 bits), 22 bits (two of 11), 25 bits (three of 9, 8, 8)."""
    rng = np.random.default_rng(n_vert)
    conn = rng.integers(0, n_vert, size=(40_000, 3)).astype(np.int32)
    conn[:50, 0] = n_vert - 1  # the largest id takes part
    print(f"[wide] boundary n_vert={n_vert}", flush=True)
    assert_same(gpu_csr("elem", conn, 0, n_vert, options=WIDE), oracle_mod.elem_neighbors(conn, 0, n_vert),
                "wide boundary elem")


def test_wide_equals_narrow_on_a_large_grid():
    """A 1024^2 coin-flip triangle grid (about 2.1 M triangles, 20 vertex
    bits): the 11-bit and 8-bit element sorts give the same bytes."""
    m = mg.tri_grid(1024, diag="coin", seed=41)
    print(f"[wide] {m.name} n_elem={m.n_elem}", flush=True)
    wide = gpu_csr("both", m.conn, m.etype, m.n_vert, options=WIDE)
    narrow = gpu_csr("both", m.conn, m.etype, m.n_vert, options={"digit_bits": 8})
    for (a, b), rel in zip(zip(wide, narrow), ("node", "elem")):
        assert_same(a, b, f"wide vs narrow {rel}")


def test_wide_mixed_mesh(oracle_mod):
    from tests.test_gpu_mixed import gpu_mixed
    mm = mg.random_mixed(30_000, 100_000, seed=77)
    print(f"[wide] mixed n_elem={mm.etypes.size}", flush=True)
    (nr, nc), (er, ec) = gpu_mixed(mm.conn, mm.etypes, mm.n_vert, options=WIDE)
    assert_same((er, ec), oracle_mod.mixed_elem_neighbors(mm.conn, mm.etypes, mm.n_vert), "wide mixed elem")
    assert_same((nr, nc), oracle_mod.mixed_node_neighbors(mm.conn, mm.etypes, mm.n_vert), "wide mixed node")
