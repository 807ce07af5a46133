// Host-side interface between the C ABI and the two pipelines.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mesh_neighbors.h"

namespace mnb {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// ---- node pipeline ---------------------------------------------------------
struct NodePlan {
    int64_t n_elem = 0;
    int32_t etype = 0;
    int32_t n_vert = 0;
    int64_t n_pairs = 0;      // 2 * edges per element * n_elem
    uint32_t id_bits = 1;     // b: bits of a vertex id in the packed key
    int n_pass = 0;           // radix passes over the 2b key bits (full-key mode)
    uint32_t hi_bits = 1;     // vertex-rows mode: bits sorted above the low b bits
    int n_pass_rows = 0;      // vertex-rows mode: radix passes
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
    size_t zero_bytes = 0;    // bytes from 0 cleared at the start of a call
    size_t total = 0;
};

bool plan_node(int64_t n_elem, int32_t etype, int32_t n_vert, NodePlan* p);
hipError_t run_node(const NodePlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols,
                    int64_t cols_capacity, void* ws, hipStream_t stream);

// ---- element pipeline --------------------------------------------------------
struct ElemPlan {
    int64_t n_elem = 0;
    int32_t etype = 0;
    int32_t n_vert = 0;
    int64_t n_slots = 0;      // npe * n_elem (pairs before dropping repeats)
    uint32_t id_bits = 1;     // bits of a vertex id
    int n_pass = 0;           // radix passes over the vertex bits
    int64_t n_tiles = 0;      // radix tiles (room for any tile shape)
    size_t off_hist = 0, off_lb0 = 0, off_lb1 = 0, off_keys0 = 0, off_keys1 = 0;
    size_t off_bmin = 0;      // block minima of the row-start fill
    size_t zero_bytes = 0;
    size_t total = 0;
};

bool plan_elem(int64_t n_elem, int32_t etype, int32_t n_vert, ElemPlan* p);
hipError_t run_elem(const ElemPlan& p, const int32_t* conn, int32_t* row_ptr, int32_t* cols,
                    int64_t cols_capacity, void* ws, hipStream_t stream);

// ---- batched pipelines -------------------------------------------------------
struct BatchPlan {
    int64_t n_keys = 0;       // directed pairs (node) or connectivity slots (element)
    uint32_t digit_bits = 0;  // key bits the radix passes cover
    int n_pass = 0;
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
};

bool plan_batch(int64_t n_keys, uint32_t digit_bits, int32_t rows_vert, int32_t total_vert, BatchPlan* p);
uint32_t batch_node_lo_bits(int32_t max_vert);
uint32_t batch_hi_bits(int32_t total_vert);
hipError_t run_batch_node(const BatchPlan& p, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                          uint32_t lo_bits, int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                          void* ws, hipStream_t s);
hipError_t run_batch_elem(const BatchPlan& p, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                          int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap, void* ws,
                          hipStream_t s);

// Node algorithm (process-wide): 0 = LSD sort of the full key, then one
// unique/CSR pass; 1 = LSD sort of the vertex bits only, then per-row sort
// and deduplication in LDS, scan and gather; 2 = each element edge once,
// keyed by its lower vertex, rows deduplicated, the unique edges transposed
// and sorted by their higher vertex, both halves merged per row.
int node_sort_mode();

// Clears `bytes` (a multiple of 4) from `p` with a fill kernel (no memset
// nodes, so the sequence can be captured into a graph).
hipError_t zero_words(void* p, size_t bytes, hipStream_t stream);
hipError_t fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t stream);

// Several fills (32-bit words, each region its own value) in one launch.
constexpr int MAX_FILL_REGIONS = 3;
struct FillRegion {
    void* p;
    int64_t n_words;
    uint32_t value;
};
hipError_t fill_regions(const FillRegion* r, int count, hipStream_t stream);

}  // namespace mnb
