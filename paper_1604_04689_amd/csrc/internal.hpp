// Host-side interface between the C ABI and the pipelines.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mesh_neighbors.h"

namespace mnb {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Node algorithms (mesh_node_sort).
enum NodeSort : int { NS_FULL_KEY = 0, NS_VERTEX_ROWS = 1, NS_EDGE_ROWS = 2, NS_ELEM_ROWS = 3 };

// Options of one call with the defaults filled in.
struct Opts {
    int node_sort = NS_ELEM_ROWS;
    int shape = 0;       // requested radix tile shape
    int digit_bits = -1;  // requested radix digit width (-1: the rule for the sort at hand)
    int64_t chunk_keys = 0;  // bounded-memory build: pairs sorted at once (0: the whole mesh)
};

// false: an option out of range (MESH_ERR_INVALID_ARG).  chunk_keys > 0 is an
// option only where allow_chunk is set (single-mesh calls).
bool resolve_options(const mesh_options* o, Opts* out, bool allow_chunk = false);

// Smallest b >= 1 with 2^b >= n.
uint32_t bits_for_count(int64_t n);
// Bits of a vertex id in [0, n_vert): bits of n_vert - 1 (at least 1).
uint32_t id_bits_for(int32_t n_vert);

// ---- sort plan shared by the radix pipelines ---------------------------------
// Digit passes over `bits` key bits: the widths of each pass, low digit
// first.  8-bit passes (radix_pass), or, when `wide`, passes of up to 11 bits
// (radix_wide_pass) with the bits split as evenly as the pass count allows.
struct PassPlan {
    int n_pass = 0;
    bool wide = false;
    uint32_t width[8] = {};  // digit width of each pass
    uint32_t shift[8] = {};  // first key bit of each pass, relative to the sorted field
    // histogram words per pass (the digit values of the widest pass)
    uint32_t hist_stride() const { return wide ? 2048u : 256u; }
};
// digit_bits 8: 8-bit passes; 11: passes of up to 11 bits when that takes
// fewer passes than 8-bit ones (else 8-bit passes).
PassPlan plan_passes(uint32_t bits, int digit_bits);
// The element sort's digit width when the options leave it open (8: the
// wide pass is slower on every mesh measured; it stays selectable).
int default_elem_digit_bits(uint32_t id_bits, int64_t n_keys);

// ---- element pipeline --------------------------------------------------------
struct ElemPlan {
    int64_t n_elem = 0;
    int32_t etype = 0;
    int32_t n_vert = 0;
    int64_t n_slots = 0;      // npe * n_elem (pairs before dropping repeats)
    uint32_t id_bits = 1;     // bits of a vertex id
    PassPlan pp;              // radix passes over the vertex bits
    int64_t n_tiles = 0;      // radix tiles (room for any tile shape)
    size_t off_hist = 0, off_lb0 = 0, off_lb1 = 0, off_keys0 = 0, off_keys1 = 0;
    size_t off_bmin = 0;      // block minima of the row-start fill
    size_t off_part = 0;      // wide passes: block partials of the histograms
    size_t zero_bytes = 0;
    size_t total = 0;
    Opts opts;
};

struct FillRegion;
bool plan_elem(int64_t n_elem, int32_t etype, int32_t n_vert, const Opts& o, ElemPlan* p, size_t base = 0);
// The element sort over n_slots (vertex, element) slots (meshes of several types).
bool plan_elem_slots(int64_t n_slots, int32_t n_vert, const Opts& o, ElemPlan* p);
// extra: one more region cleared by the call's fill launch (may be null).
hipError_t run_elem(const ElemPlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols,
                    int64_t cols_capacity, void* ws, hipStream_t stream, bool keep_err = false,
                    const FillRegion* extra = nullptr);

// ---- node relation through the element rows (ELEM_ROWS) ------------------------
// Work of the gather/dedup stage after the element relation: tiles of
// ER_TILE element-CSR entries, each row's distinct count, the rows' values
// staged at S slots per entry, and the look-back words of the count scan.
struct ErowsPlan {
    int64_t n_entries = 0;    // upper bound of element-relation entries
    int slots = 0;            // candidate slots per entry (S)
    int64_t n_tiles = 0;
    int64_t long_cap = 0;
    size_t off_lb = 0;        // count scan look-back words (cleared by the call's fill)
    int64_t lb_words = 0;     // their size in 32-bit words
    size_t off_tf = 0;        // first owned vertex of every tile
    size_t off_tc = 0;        // accessor context (mesh in a batch) of that vertex
    size_t off_list = 0;      // long rows
    size_t off_deg = 0;       // distinct count of every row (n_vert + 1 ints)
    size_t off_soff = 0;      // stage offset of every row (n_vert + 1 int16)
    size_t off_temp = 0;      // staged values: S * n_entries ints
    size_t temp_bytes = 0;
};
// Sizes the stage at `off` onward; temp may alias a dead region of `alias_bytes`
// at `alias_off` when that is large enough.  Returns the end offset.
size_t plan_erows(int64_t n_entries, int slots, int32_t n_vert, size_t off, size_t alias_off, size_t alias_bytes,
                  ErowsPlan* p);

// ---- node pipeline ---------------------------------------------------------
struct NodePlan {
    int64_t n_elem = 0;
    int32_t etype = 0;
    int32_t n_vert = 0;
    int mode = 0;             // NodeSort
    int64_t n_pairs = 0;      // 2 * edges per element * n_elem
    int64_t n_keys = 0;       // keys of the first sort: n_pairs, or n_edges under EDGE_ROWS
    uint32_t id_bits = 1;     // b: bits of a vertex id in the packed key
    PassPlan pp;              // radix passes (over 2b bits, or the vertex bits)
    uint32_t sort_bits = 0;   // bits the first sort covers
    int64_t n_tiles = 0;      // radix tiles
    int64_t n_utiles = 0;     // unique/CSR tiles
    int64_t long_cap = 0;     // vertex-rows mode: capacity of the long-row list
    // workspace offsets (bytes)
    size_t off_hist = 0, off_ulb = 0, off_lb0 = 0, off_lb1 = 0, off_keys0 = 0, off_keys1 = 0;
    size_t off_deg = 0, off_src = 0, off_long = 0;
    int64_t n_edges = 0;      // edge-rows mode: canonical keys (one per element edge)
    size_t off_hist2 = 0;     // edge-rows mode: digit histograms of the transposed edges
    size_t off_up = 0, off_low = 0;  // edge-rows mode: starts of higher and lower neighbours
    size_t off_bmin = 0;      // edge-rows mode: block minima of the lower-group fill
    // ELEM_ROWS: the element relation (its own plan) and, for a node-only call,
    // its CSR inside the workspace
    ElemPlan ep;
    bool internal_elem = false;
    size_t off_erp = 0, off_ecols = 0;
    ErowsPlan er;
    size_t zero_bytes = 0;    // bytes from 0 cleared at the start of a call
    size_t total = 0;
    Opts opts;
};

// internal_elem: ELEM_ROWS keeps the element CSR in the workspace (node-only
// calls); otherwise the caller's element outputs are used.
bool plan_node(int64_t n_elem, int32_t etype, int32_t n_vert, const Opts& o, bool internal_elem, NodePlan* p);
hipError_t run_node(const NodePlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                    void* ws, hipStream_t stream, bool keep_err = false, const int32_t* elem_row_ptr = nullptr,
                    const int32_t* elem_cols = nullptr, int64_t elem_cap = 0);

// ELEM_ROWS stage for one mesh of one type: node CSR from the element CSR.
hipError_t run_erows_uniform(int32_t etype, const ErowsPlan& er, const int32_t* conn, int64_t n_elem,
                             int32_t n_vert, const int32_t* erp, const int32_t* ecols, int64_t ecap,
                             int32_t* row_ptr, int32_t* cols, int64_t cols_cap, char* ws, uint32_t* err,
                             uint32_t* ticket, hipStream_t s);

// ---- bounded-memory build (chunk_keys) ------------------------------------------
// The relations of one mesh of one type, one vertex range at a time: a
// histogram over the top vertex bits (coarse bins) is read back, the host cuts
// the vertices into ranges of at most `cap` pairs and `cap` vertices, and each
// range compacts its own pairs out of the connectivity, sorts them and writes
// its rows.  Workspace: the header, the per-range histograms, the node
// stage's scan look-back, the compaction's look-back (one word per 24576
// connectivity slots) and the first pass's (all cleared per range), the
// other passes' look-back and two key buffers of cap keys, the range's
// element row starts (and, for a node-only call, its element columns), the
// coarse bins and their block partials, and the node stage's buffers for cap
// entries.
constexpr int64_t CHUNK_MIN_KEYS = 4096;
struct ChunkPlan {
    int64_t n_elem = 0;
    int32_t etype = 0;
    int32_t n_vert = 0;
    int64_t n_slots = 0;
    int64_t cap = 0;
    uint32_t coarse_bits = 0;  // vertex bits of a bin index (the top ones)
    uint32_t coarse_shift = 0; // low vertex bits inside a bin
    bool node = false;         // the node relation is written
    bool elem_out = false;     // the element relation goes to the caller
    size_t off_hist = 0, zero_bytes = 0;  // [0, zero_bytes): cleared per range (error word kept)
    size_t off_clb = 0;        // look-back words of the compaction (one per tile of slots)
    size_t off_lb0 = 0, off_lb1 = 0;
    size_t off_keys0 = 0, off_keys1 = 0, off_bmin = 0, off_erp = 0, off_ecols = 0;
    size_t off_bins = 0, off_part = 0;
    ErowsPlan er;
    size_t total = 0;
    Opts opts;
};
// false: the options do not allow a bounded-memory build of these sizes
// (MESH_ERR_INVALID_ARG).
bool plan_chunked(int64_t n_elem, int32_t etype, int32_t n_vert, const Opts& o, bool node, bool elem_out,
                  ChunkPlan* p);
// Waits on the stream once (the coarse histogram).  The element outputs may
// be null when !p.elem_out, the node outputs when !p.node.
mesh_status run_chunked(const ChunkPlan& p, const int32_t* conn, int32_t* node_row_ptr, int32_t* node_cols,
                        int64_t node_cap, int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cap, void* ws,
                        hipStream_t s);

// ---- meshes of several element types -----------------------------------------
struct MixedPlan {
    int64_t n_elem = 0, n_ids = 0, n_pairs = 0;
    int32_t n_vert = 0;
    size_t off_map = 0;       // element of every slot (n_ids ints)
    ElemPlan ep;              // the element sort over n_ids slots
    ErowsPlan er;
    size_t zero_bytes = 0;
    size_t total = 0;
    Opts opts;
};
bool plan_mixed(int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert, const Opts& o, MixedPlan* p);
hipError_t run_mixed(const MixedPlan& p, const int32_t* conn, const int32_t* elem_off, const uint8_t* etypes,
                     int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cap, int32_t* elem_row_ptr,
                     int32_t* elem_cols, int64_t elem_cap, void* ws, hipStream_t s);

// ---- batched pipelines -------------------------------------------------------
struct BatchPlan {
    int64_t n_keys = 0;       // directed pairs (node) or connectivity slots (element)
    uint32_t digit_bits = 0;  // key bits the radix passes cover
    PassPlan pp;
    int64_t n_tiles = 0, n_utiles = 0;
    size_t off_hist = 0, off_ulb = 0, off_lb0 = 0, off_lb1 = 0, off_keys0 = 0, off_keys1 = 0;
    int64_t n_lut = 0;      // segment lookup entries (one per 2^SEG_LUT_SHIFT keys, plus one)
    size_t off_lut = 0;
    size_t off_tiles = 0;   // one record per radix tile
    int32_t rows_vert = 0;  // node relation: vertices of the vertex-rows stage (0: no such stage)
    int64_t long_cap = 0;
    size_t off_deg = 0, off_src = 0, off_long = 0;
    size_t off_hist2 = 0, off_up = 0, off_low = 0;  // node relation, edge-rows algorithm
    size_t off_bmin = 0;    // block minima of a row-start fill (element rows, lower groups)
    size_t zero_bytes = 0;
    size_t total = 0;
    Opts opts;
};

// The batch plans of each call kind.
struct BatchNodePlan {
    int mode = 0;
    BatchPlan bp;             // the sort (pairs, or the element slots under ELEM_ROWS)
    bool internal_elem = false;
    size_t off_erp = 0, off_ecols = 0;
    ErowsPlan er;
    size_t off_tlists = 0;    // ELEM_ROWS: the stage's tile lists by element type
    int64_t tlist_stride = 0; // entries per list
    size_t total = 0;
};
bool plan_batch_sort(int64_t n_keys, uint32_t digit_bits, int32_t rows_vert, int32_t total_vert, const Opts& o,
                     BatchPlan* p);
bool plan_batch_elem(int64_t total_slots, int32_t total_vert, const Opts& o, BatchPlan* p, size_t base = 0);
bool plan_batch_node(int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert, const Opts& o,
                     bool internal_elem, BatchNodePlan* p);
uint32_t batch_node_lo_bits(int32_t max_vert);
hipError_t run_batch_node(const BatchNodePlan& p, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                          uint32_t lo_bits, int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                          void* ws, hipStream_t s, bool keep_err = false, const int32_t* elem_row_ptr = nullptr,
                          const int32_t* elem_cols = nullptr, int64_t elem_cap = 0);
hipError_t run_batch_elem(const BatchPlan& p, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                          int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap, void* ws,
                          hipStream_t s, bool keep_err = false, const FillRegion* extra = nullptr);

// Clears `bytes` (a multiple of 4) from `p` with a fill kernel (no memset
// nodes, so the sequence can be captured into a graph).
hipError_t zero_words(void* p, size_t bytes, hipStream_t stream);
hipError_t fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t stream);

// Several fills (32-bit words, each region its own value) in one launch.
constexpr int MAX_FILL_REGIONS = 4;
struct FillRegion {  // (declared above)
    void* p;
    int64_t n_words;
    uint32_t value;
};
hipError_t fill_regions(const FillRegion* r, int count, hipStream_t stream);

// Device address of the fixed scratch array of mesh_neighbors_noalloc on the
// current device (looked up once per device).
hipError_t noalloc_scratch(void** out);

// The workspace's first word is the error word; keep_err leaves it (and only
// it) untouched when the header is cleared, for a second pipeline in the same
// call.
inline FillRegion header_fill(void* ws, size_t zero_bytes, bool keep_err) {
    char* w = (char*)ws;
    return keep_err ? FillRegion{w + 4, (int64_t)(zero_bytes / 4) - 1, 0u} : FillRegion{ws, (int64_t)(zero_bytes / 4), 0u};
}

}  // namespace mnb
