// C ABI of the one-ring neighbor library: argument checks, workspace sizing
// and dispatch to the node and element pipelines.  Declared in
// include/mesh_neighbors.h.
#include <climits>

#include "../../include/mesh_neighbors.h"
#include "common.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "radix.hpp"

namespace mnb {

constexpr int FILL_BLOCK = 256;
constexpr int FILL_GRID_MAX = 4096;

__global__ __launch_bounds__(FILL_BLOCK) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t value) {
    for (int64_t i = (int64_t)blockIdx.x * FILL_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * FILL_BLOCK)
        p[i] = value;
}

static hipError_t fill_words(uint32_t* p, int64_t n, uint32_t value, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)tmin<int64_t>(ceil_div(n, FILL_BLOCK), FILL_GRID_MAX);
    return launch("fill", fill_u32_kernel, dim3(grid), dim3(FILL_BLOCK), s, p, n, value);
}

hipError_t zero_words(void* p, size_t bytes, hipStream_t s) {
    return fill_words((uint32_t*)p, (int64_t)(bytes / 4), 0u, s);
}

hipError_t fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s) {
    return fill_words((uint32_t*)p, n, (uint32_t)value, s);
}

// Up to MAX_FILL_REGIONS regions, each with its own value, in one launch.
struct FillSet {
    uint32_t* p[MAX_FILL_REGIONS];
    int64_t end[MAX_FILL_REGIONS];  // running word counts
    uint32_t value[MAX_FILL_REGIONS];
    int count;
};

__global__ __launch_bounds__(FILL_BLOCK) void fill_set_kernel(FillSet f) {
    const int64_t total = f.end[f.count - 1];
    for (int64_t i = (int64_t)blockIdx.x * FILL_BLOCK + threadIdx.x; i < total; i += (int64_t)gridDim.x * FILL_BLOCK) {
        int k = 0;
        while (i >= f.end[k]) ++k;
        f.p[k][i - (k ? f.end[k - 1] : 0)] = f.value[k];
    }
}

hipError_t fill_regions(const FillRegion* r, int count, hipStream_t s) {
    FillSet f{};
    int64_t total = 0;
    for (int i = 0; i < count && i < MAX_FILL_REGIONS; ++i) {
        if (r[i].n_words <= 0) continue;
        f.p[f.count] = (uint32_t*)r[i].p;
        total += r[i].n_words;
        f.end[f.count] = total;
        f.value[f.count] = r[i].value;
        ++f.count;
    }
    if (f.count == 0) return hipSuccess;
    const int grid = (int)tmin<int64_t>(ceil_div(total, FILL_BLOCK), FILL_GRID_MAX);
    return launch("fill", fill_set_kernel, dim3(grid), dim3(FILL_BLOCK), s, f);
}

bool resolve_options(const mesh_options* o, Opts* out, bool allow_chunk) {
    Opts r;
    if (o) {
        if (o->node_sort < -1 || o->node_sort > NS_ELEM_ROWS) return false;
        if (o->radix_shape < -1 || o->radix_shape >= N_RADIX_SHAPES) return false;
        if (o->digit_bits != -1 && o->digit_bits != 8 && o->digit_bits != 11) return false;
        if (o->chunk_keys < -1 || (o->chunk_keys > 0 && (!allow_chunk || o->chunk_keys < CHUNK_MIN_KEYS)))
            return false;
        if (o->node_sort >= 0) r.node_sort = o->node_sort;
        if (o->radix_shape >= 0) r.shape = o->radix_shape;
        r.digit_bits = o->digit_bits;
        r.chunk_keys = o->chunk_keys > 0 ? o->chunk_keys : 0;
    }
    *out = r;
    return true;
}

uint32_t bits_for_count(int64_t n) {
    uint32_t b = 1;
    while (b < 62 && ((int64_t)1 << b) < n) ++b;
    return b;
}

uint32_t id_bits_for(int32_t n_vert) { return bits_for_count(n_vert); }

PassPlan plan_passes(uint32_t bits, int digit_bits) {
    PassPlan pp;
    const int narrow = (int)ceil_div(bits, RBITS);
    const int wide = (int)ceil_div(bits, WBITS);
    if (digit_bits == WBITS && wide < narrow) {
        // as even a split as the pass count allows: the narrowest digits keep
        // the longest runs per tile (better coalesced writes)
        pp.wide = true;
        pp.n_pass = wide;
        uint32_t at = 0;
        for (int q = 0; q < wide; ++q) {
            const uint32_t w = bits / (uint32_t)wide + ((uint32_t)q < bits % (uint32_t)wide ? 1u : 0u);
            pp.shift[q] = at;
            pp.width[q] = w;
            at += w;
        }
        return pp;
    }
    pp.n_pass = narrow;
    for (int q = 0; q < pp.n_pass && q < 8; ++q) {
        pp.shift[q] = (uint32_t)q * RBITS;
        pp.width[q] = tmin<uint32_t>(RBITS, bits - (uint32_t)q * RBITS);
    }
    return pp;
}

int default_elem_digit_bits(uint32_t, int64_t) {
    // Measured on MI355X: two 11-bit passes over the 22 vertex bits of an
    // 8.4 M-triangle mesh took 345 + 438 us against 137 + 139 + 139 us for
    // three 8-bit ones (2048 digits of an 8192-key tile average 4 keys each:
    // look-back words cost about 3/4 of the key traffic and writes come in
    // 32-byte runs), so the rule keeps 8-bit passes.
    return RBITS;
}

}  // namespace mnb

using namespace mnb;

static bool aligned(const void* p) { return ((uintptr_t)p % ALIGN) == 0; }

static mesh_status check_sizes(int64_t n_elem, int32_t etype, int32_t n_vert) {
    if (n_elem < 0 || n_vert < 0) return MESH_ERR_INVALID_ARG;
    if (nodes_per_elem(etype) == 0) return MESH_ERR_UNSUPPORTED_TYPE;
    return MESH_OK;
}

// Output pointers of one relation: row_ptr always, cols when the capacity is
// positive.
static bool outputs_ok(const int32_t* row_ptr, const int32_t* cols, int64_t cap) {
    return row_ptr && cap >= 0 && (cap == 0 || cols);
}

static mesh_status workspace_ok(const void* ws, size_t bytes, size_t need) {
    if (!ws) return MESH_ERR_INVALID_ARG;
    return bytes < need || !aligned(ws) ? MESH_ERR_WORKSPACE : MESH_OK;
}

// Plans of one single-mesh call (both relations planned; node-only and
// element-only calls use one of them).
struct SinglePlans {
    Opts o;
    NodePlan node;
    ElemPlan elem;
    bool chunked = false;  // bounded-memory build (chunk_keys): `chunk` runs the call
    ChunkPlan chunk;
};

enum Relations { REL_NODE = 1, REL_ELEM = 2, REL_BOTH = 3 };

static mesh_status plan_single(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                               int relations, bool node_internal_elem, SinglePlans* sp) {
    mesh_status st = check_sizes(n_elem, etype, n_vert);
    if (st != MESH_OK) return st;
    if (!resolve_options(opts, &sp->o, /*allow_chunk=*/true)) return MESH_ERR_INVALID_ARG;
    // the relation's keys below 2^31: directed pairs for the node relation
    // (the larger count), node slots for the element relation alone
    if ((relations & REL_NODE) && n_elem > INT32_MAX / (2 * edges_per_elem(etype))) return MESH_ERR_OVERFLOW;
    if (n_elem > INT32_MAX / nodes_per_elem(etype)) return MESH_ERR_OVERFLOW;
    if ((relations & REL_NODE) && !plan_node(n_elem, etype, n_vert, sp->o, node_internal_elem, &sp->node))
        return MESH_ERR_INVALID_ARG;
    if (!plan_elem(n_elem, etype, n_vert, sp->o, &sp->elem)) return MESH_ERR_INVALID_ARG;
    if (sp->o.chunk_keys > 0) {
        sp->chunked = true;
        if (!plan_chunked(n_elem, etype, n_vert, sp->o, (relations & REL_NODE) != 0, (relations & REL_ELEM) != 0,
                          &sp->chunk))
            return MESH_ERR_INVALID_ARG;
    }
    return MESH_OK;
}

static mesh_status hip_status(hipError_t e) { return e == hipSuccess ? MESH_OK : MESH_ERR_HIP; }

extern "C" {

int32_t mesh_abi_version(void) { return (2 << 16) | 3; }

mesh_options mesh_default_options(void) {
    mesh_options o;
    o.node_sort = -1;
    o.radix_shape = -1;
    o.digit_bits = -1;
    o.chunk_keys = -1;
    for (int i = 0; i < 4; ++i) o.reserved[i] = 0;
    return o;
}

const char* mesh_status_string(mesh_status s) {
    switch (s) {
        case MESH_OK: return "ok";
        case MESH_ERR_INVALID_ARG: return "invalid argument";
        case MESH_ERR_UNSUPPORTED_TYPE: return "unsupported element type";
        case MESH_ERR_WORKSPACE: return "workspace too small or misaligned";
        case MESH_ERR_CAPACITY: return "cols capacity too small";
        case MESH_ERR_OVERFLOW: return "size beyond the supported range";
        case MESH_ERR_INDEX_RANGE: return "vertex id outside [0, n_vert)";
        case MESH_ERR_HIP: return "HIP runtime error";
        case MESH_ERR_INTERNAL: return "internal device check failed";
        case MESH_ERR_SCRATCH_LIMIT: return "mesh needs more scratch than the fixed no-allocation array holds";
        case MESH_ERR_CHUNK: return "a vertex bin holds more pairs than chunk_keys";
    }
    return "unknown status";
}

// ---- single meshes ------------------------------------------------------------

mesh_status mesh_node_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                                      size_t* workspace_bytes, int64_t* cols_capacity) {
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    SinglePlans sp;
    mesh_status st = plan_single(n_elem, etype, n_vert, opts, REL_NODE, true, &sp);
    if (st != MESH_OK) return st;
    *workspace_bytes = sp.chunked ? sp.chunk.total : sp.node.total;
    *cols_capacity = sp.node.n_pairs;
    return MESH_OK;
}

mesh_status mesh_node_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                int32_t* row_ptr, int32_t* cols, int64_t cols_capacity, const mesh_options* opts,
                                void* workspace, size_t workspace_bytes, void* stream) {
    SinglePlans sp;
    mesh_status st = plan_single(n_elem, etype, n_vert, opts, REL_NODE, true, &sp);
    if (st != MESH_OK) return st;
    if ((n_elem > 0 && !conn) || !outputs_ok(row_ptr, cols, cols_capacity)) return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, sp.chunked ? sp.chunk.total : sp.node.total);
    if (st != MESH_OK) return st;
    if (sp.chunked)
        return run_chunked(sp.chunk, conn, row_ptr, cols, cols_capacity, nullptr, nullptr, 0, workspace,
                           (hipStream_t)stream);
    return hip_status(run_node(sp.node, conn, row_ptr, cols, cols_capacity, workspace, (hipStream_t)stream));
}

mesh_status mesh_elem_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                                      size_t* workspace_bytes, int64_t* cols_capacity) {
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    SinglePlans sp;
    mesh_status st = plan_single(n_elem, etype, n_vert, opts, REL_ELEM, true, &sp);
    if (st != MESH_OK) return st;
    *workspace_bytes = sp.chunked ? sp.chunk.total : sp.elem.total;
    *cols_capacity = sp.elem.n_slots;
    return MESH_OK;
}

mesh_status mesh_elem_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                int32_t* row_ptr, int32_t* cols, int64_t cols_capacity, const mesh_options* opts,
                                void* workspace, size_t workspace_bytes, void* stream) {
    SinglePlans sp;
    mesh_status st = plan_single(n_elem, etype, n_vert, opts, REL_ELEM, true, &sp);
    if (st != MESH_OK) return st;
    if ((n_elem > 0 && !conn) || !outputs_ok(row_ptr, cols, cols_capacity)) return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, sp.chunked ? sp.chunk.total : sp.elem.total);
    if (st != MESH_OK) return st;
    if (sp.chunked)
        return run_chunked(sp.chunk, conn, nullptr, nullptr, 0, row_ptr, cols, cols_capacity, workspace,
                           (hipStream_t)stream);
    return hip_status(run_elem(sp.elem, conn, row_ptr, cols, cols_capacity, workspace, (hipStream_t)stream));
}

// Both relations: under ELEM_ROWS the node plan already holds the element
// sort (the element CSR goes to the caller's outputs); otherwise the two
// pipelines share one workspace, one after the other.
static size_t both_bytes(const SinglePlans& sp) {
    if (sp.chunked) return sp.chunk.total;
    if (sp.node.mode == NS_ELEM_ROWS) return sp.node.total;
    return sp.node.total > sp.elem.total ? sp.node.total : sp.elem.total;
}

mesh_status mesh_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, const mesh_options* opts,
                                 size_t* workspace_bytes, int64_t* node_cols_capacity,
                                 int64_t* elem_cols_capacity) {
    if (!workspace_bytes || !node_cols_capacity || !elem_cols_capacity) return MESH_ERR_INVALID_ARG;
    SinglePlans sp;
    mesh_status st = plan_single(n_elem, etype, n_vert, opts, REL_BOTH, false, &sp);
    if (st != MESH_OK) return st;
    *workspace_bytes = both_bytes(sp);
    *node_cols_capacity = sp.node.n_pairs;
    *elem_cols_capacity = sp.elem.n_slots;
    return MESH_OK;
}

mesh_status mesh_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                           int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                           int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                           const mesh_options* opts, void* workspace, size_t workspace_bytes, void* stream) {
    SinglePlans sp;
    mesh_status st = plan_single(n_elem, etype, n_vert, opts, REL_BOTH, false, &sp);
    if (st != MESH_OK) return st;
    if ((n_elem > 0 && !conn) || !outputs_ok(node_row_ptr, node_cols, node_cols_capacity) ||
        !outputs_ok(elem_row_ptr, elem_cols, elem_cols_capacity))
        return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, both_bytes(sp));
    if (st != MESH_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (sp.chunked)
        return run_chunked(sp.chunk, conn, node_row_ptr, node_cols, node_cols_capacity, elem_row_ptr, elem_cols,
                           elem_cols_capacity, workspace, s);
    if (sp.node.mode == NS_ELEM_ROWS)
        return hip_status(run_node(sp.node, conn, node_row_ptr, node_cols, node_cols_capacity, workspace, s, false,
                                   elem_row_ptr, elem_cols, elem_cols_capacity));
    hipError_t e = run_elem(sp.elem, conn, elem_row_ptr, elem_cols, elem_cols_capacity, workspace, s);
    if (e == hipSuccess)
        e = run_node(sp.node, conn, node_row_ptr, node_cols, node_cols_capacity, workspace, s, /*keep_err=*/true);
    return hip_status(e);
}

// ---- meshes of several element types -------------------------------------------

static mesh_status plan_mixed_call(int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert,
                                   const mesh_options* opts, MixedPlan* p) {
    if (n_elem < 0 || n_ids < 0 || n_pairs < 0 || n_vert < 0) return MESH_ERR_INVALID_ARG;
    Opts o;
    if (!resolve_options(opts, &o) || o.node_sort != NS_ELEM_ROWS) return MESH_ERR_INVALID_ARG;
    if (n_ids > INT32_MAX || n_pairs > INT32_MAX || n_elem > INT32_MAX) return MESH_ERR_OVERFLOW;
    if (!plan_mixed(n_elem, n_ids, n_pairs, n_vert, o, p)) return MESH_ERR_INVALID_ARG;
    return MESH_OK;
}

mesh_status mesh_mixed_neighbors_query(int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert,
                                       const mesh_options* opts, size_t* workspace_bytes,
                                       int64_t* node_cols_capacity, int64_t* elem_cols_capacity) {
    if (!workspace_bytes || !node_cols_capacity || !elem_cols_capacity) return MESH_ERR_INVALID_ARG;
    MixedPlan p;
    mesh_status st = plan_mixed_call(n_elem, n_ids, n_pairs, n_vert, opts, &p);
    if (st != MESH_OK) return st;
    *workspace_bytes = p.total;
    *node_cols_capacity = n_pairs;
    *elem_cols_capacity = n_ids;
    return MESH_OK;
}

mesh_status mesh_mixed_neighbors(const int32_t* conn, const int32_t* elem_off, const uint8_t* etypes,
                                 int64_t n_elem, int64_t n_ids, int64_t n_pairs, int32_t n_vert,
                                 int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                 int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                 const mesh_options* opts, void* workspace, size_t workspace_bytes, void* stream) {
    MixedPlan p;
    mesh_status st = plan_mixed_call(n_elem, n_ids, n_pairs, n_vert, opts, &p);
    if (st != MESH_OK) return st;
    if ((n_elem > 0 && (!elem_off || !etypes)) || (n_ids > 0 && !conn) ||
        !outputs_ok(node_row_ptr, node_cols, node_cols_capacity) ||
        !outputs_ok(elem_row_ptr, elem_cols, elem_cols_capacity))
        return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, p.total);
    if (st != MESH_OK) return st;
    return hip_status(run_mixed(p, conn, elem_off, etypes, node_row_ptr, node_cols, node_cols_capacity, elem_row_ptr,
                                elem_cols, elem_cols_capacity, workspace, (hipStream_t)stream));
}

// ---- batches ----------------------------------------------------------------------

static mesh_status batch_sizes_ok(int32_t n_mesh, int64_t total_pairs, int64_t total_slots, int32_t total_vert,
                                  int32_t max_vert) {
    if (n_mesh < 0 || total_pairs < 0 || total_slots < 0 || total_vert < 0 || max_vert < 0 || max_vert > total_vert)
        return MESH_ERR_INVALID_ARG;
    if (total_pairs > INT32_MAX || total_slots > INT32_MAX) return MESH_ERR_OVERFLOW;
    return MESH_OK;
}

struct BatchPlans {
    Opts o;
    BatchNodePlan node;
    BatchPlan elem;
};

static mesh_status plan_batch_call(int32_t n_mesh, int64_t total_pairs, int64_t total_slots, int32_t total_vert,
                                   int32_t max_vert, const mesh_options* opts, bool node_internal_elem,
                                   BatchPlans* bp) {
    mesh_status st = batch_sizes_ok(n_mesh, total_pairs, total_slots, total_vert, max_vert);
    if (st != MESH_OK) return st;
    if (!resolve_options(opts, &bp->o)) return MESH_ERR_INVALID_ARG;
    if (!plan_batch_node(total_pairs, total_slots, total_vert, max_vert, bp->o, node_internal_elem, &bp->node))
        return MESH_ERR_OVERFLOW;
    if (!plan_batch_elem(total_slots, total_vert, bp->o, &bp->elem)) return MESH_ERR_OVERFLOW;
    return MESH_OK;
}

mesh_status mesh_batch_node_neighbors_query(int32_t n_mesh, int64_t total_pairs, int64_t total_slots,
                                            int32_t total_vert, int32_t max_vert, const mesh_options* opts,
                                            size_t* workspace_bytes, int64_t* cols_capacity) {
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    BatchPlans bp;
    mesh_status st = plan_batch_call(n_mesh, total_pairs, total_slots, total_vert, max_vert, opts, true, &bp);
    if (st != MESH_OK) return st;
    *workspace_bytes = bp.node.total;
    *cols_capacity = total_pairs;
    return MESH_OK;
}

mesh_status mesh_batch_node_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                      int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert,
                                      int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                      const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                      void* stream) {
    BatchPlans bp;
    mesh_status st = plan_batch_call(n_mesh, total_pairs, total_slots, total_vert, max_vert, opts, true, &bp);
    if (st != MESH_OK) return st;
    if (((total_pairs > 0 || total_slots > 0) && (!conn || !segs)) || !outputs_ok(row_ptr, cols, cols_capacity))
        return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, bp.node.total);
    if (st != MESH_OK) return st;
    return hip_status(run_batch_node(bp.node, conn, segs, n_mesh, batch_node_lo_bits(max_vert), total_vert, row_ptr,
                                     cols, cols_capacity, workspace, (hipStream_t)stream));
}

mesh_status mesh_batch_elem_neighbors_query(int32_t n_mesh, int64_t total_slots, int32_t total_vert,
                                            const mesh_options* opts, size_t* workspace_bytes,
                                            int64_t* cols_capacity) {
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    mesh_status st = batch_sizes_ok(n_mesh, 0, total_slots, total_vert, 0);
    if (st != MESH_OK) return st;
    Opts o;
    if (!resolve_options(opts, &o)) return MESH_ERR_INVALID_ARG;
    BatchPlan p;
    if (!plan_batch_elem(total_slots, total_vert, o, &p)) return MESH_ERR_OVERFLOW;
    *workspace_bytes = p.total;
    *cols_capacity = total_slots;
    return MESH_OK;
}

mesh_status mesh_batch_elem_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                      int64_t total_slots, int32_t total_vert, int32_t* row_ptr, int32_t* cols,
                                      int64_t cols_capacity, const mesh_options* opts, void* workspace,
                                      size_t workspace_bytes, void* stream) {
    mesh_status st = batch_sizes_ok(n_mesh, 0, total_slots, total_vert, 0);
    if (st != MESH_OK) return st;
    Opts o;
    if (!resolve_options(opts, &o)) return MESH_ERR_INVALID_ARG;
    BatchPlan p;
    if (!plan_batch_elem(total_slots, total_vert, o, &p)) return MESH_ERR_OVERFLOW;
    if ((total_slots > 0 && (!conn || !segs)) || !outputs_ok(row_ptr, cols, cols_capacity))
        return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, p.total);
    if (st != MESH_OK) return st;
    return hip_status(run_batch_elem(p, conn, segs, n_mesh, total_vert, row_ptr, cols, cols_capacity, workspace,
                                     (hipStream_t)stream));
}

static size_t batch_both_bytes(const BatchPlans& bp) {
    if (bp.node.mode == NS_ELEM_ROWS) return bp.node.total;
    return bp.node.total > bp.elem.total ? bp.node.total : bp.elem.total;
}

mesh_status mesh_batch_neighbors_query(int32_t n_mesh, int64_t total_pairs, int64_t total_slots,
                                       int32_t total_vert, int32_t max_vert, const mesh_options* opts,
                                       size_t* workspace_bytes, int64_t* node_cols_capacity,
                                       int64_t* elem_cols_capacity) {
    if (!workspace_bytes || !node_cols_capacity || !elem_cols_capacity) return MESH_ERR_INVALID_ARG;
    BatchPlans bp;
    mesh_status st = plan_batch_call(n_mesh, total_pairs, total_slots, total_vert, max_vert, opts, false, &bp);
    if (st != MESH_OK) return st;
    *workspace_bytes = batch_both_bytes(bp);
    *node_cols_capacity = total_pairs;
    *elem_cols_capacity = total_slots;
    return MESH_OK;
}

mesh_status mesh_batch_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                 int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert,
                                 int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                 int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                 const mesh_options* opts, void* workspace, size_t workspace_bytes, void* stream) {
    BatchPlans bp;
    mesh_status st = plan_batch_call(n_mesh, total_pairs, total_slots, total_vert, max_vert, opts, false, &bp);
    if (st != MESH_OK) return st;
    if (((total_pairs > 0 || total_slots > 0) && (!conn || !segs)) ||
        !outputs_ok(node_row_ptr, node_cols, node_cols_capacity) ||
        !outputs_ok(elem_row_ptr, elem_cols, elem_cols_capacity))
        return MESH_ERR_INVALID_ARG;
    st = workspace_ok(workspace, workspace_bytes, batch_both_bytes(bp));
    if (st != MESH_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t lo = batch_node_lo_bits(max_vert);
    if (bp.node.mode == NS_ELEM_ROWS)
        return hip_status(run_batch_node(bp.node, conn, segs, n_mesh, lo, total_vert, node_row_ptr, node_cols,
                                         node_cols_capacity, workspace, s, false, elem_row_ptr, elem_cols,
                                         elem_cols_capacity));
    hipError_t e = run_batch_elem(bp.elem, conn, segs, n_mesh, total_vert, elem_row_ptr, elem_cols,
                                  elem_cols_capacity, workspace, s);
    if (e == hipSuccess)
        e = run_batch_node(bp.node, conn, segs, n_mesh, lo, total_vert, node_row_ptr, node_cols, node_cols_capacity,
                           workspace, s, /*keep_err=*/true);
    return hip_status(e);
}

// ---- tuning information and diagnostics ---------------------------------------------

int32_t mesh_radix_shape_count(void) { return N_RADIX_SHAPES; }

mesh_status mesh_radix_shape_info(int32_t shape, int32_t* block, int32_t* items) {
    if (shape < 0 || shape >= N_RADIX_SHAPES || !block || !items) return MESH_ERR_INVALID_ARG;
    *block = RADIX_SHAPES[shape].block;
    *items = RADIX_SHAPES[shape].items;
    return MESH_OK;
}

mesh_status mesh_radix_launch_shape(int32_t shape, int32_t digit_bits, int64_t n_keys, int32_t* block,
                                    int32_t* items, int32_t* bits) {
    if (!block || !items || !bits || n_keys < 0) return MESH_ERR_INVALID_ARG;
    mesh_options o = mesh_default_options();
    o.radix_shape = shape;
    o.digit_bits = digit_bits;
    Opts r;
    if (!resolve_options(&o, &r)) return MESH_ERR_INVALID_ARG;
    const int eff = radix_effective_shape(r.shape, n_keys);
    if (r.digit_bits == WBITS && n_keys < LB32_MAX_KEYS) {  // the wide pass has one tile shape
        *block = WIDE_BLOCK;
        *items = WIDE_ITEMS;
        *bits = WBITS;
        return MESH_OK;
    }
    *block = RADIX_SHAPES[eff].block;
    *items = RADIX_SHAPES[eff].items;
    *bits = RBITS;
    return MESH_OK;
}

mesh_status mesh_check(const void* workspace, void* stream) {
    if (!workspace) {  // the fixed scratch of mesh_neighbors_noalloc on the current device
        void* p = nullptr;
        if (noalloc_scratch(&p) != hipSuccess) return MESH_ERR_HIP;
        workspace = p;
    }
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MESH_ERR_HIP;
    uint32_t err = 0;
    if (hipMemcpy(&err, workspace, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return MESH_ERR_HIP;
    if (err & ERR_INTERNAL) return MESH_ERR_INTERNAL;
    if (err & ERR_INDEX_RANGE) return MESH_ERR_INDEX_RANGE;
    if (err & ERR_CAPACITY) return MESH_ERR_CAPACITY;
    return MESH_OK;
}

}  // extern "C"
