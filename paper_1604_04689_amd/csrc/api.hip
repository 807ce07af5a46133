// C ABI of the one-ring neighbor library: argument checks, workspace sizing
// and dispatch to the node and element pipelines.  Declared in
// include/mesh_neighbors.h.
#include <atomic>
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

static std::atomic<int> g_radix_shape{DEFAULT_RADIX_SHAPE};
static std::atomic<int> g_node_sort{0};

int node_sort_mode() { return g_node_sort.load(std::memory_order_relaxed); }

int radix_shape() { return g_radix_shape.load(std::memory_order_relaxed); }

}  // namespace mnb

using namespace mnb;

static bool aligned(const void* p) { return ((uintptr_t)p % ALIGN) == 0; }

static mesh_status check_sizes(int64_t n_elem, int32_t etype, int32_t n_vert) {
    if (n_elem < 0 || n_vert < 0) return MESH_ERR_INVALID_ARG;
    if (nodes_per_elem(etype) == 0) return MESH_ERR_UNSUPPORTED_TYPE;
    return MESH_OK;
}

extern "C" {

int32_t mesh_abi_version(void) { return (1 << 16) | 0; }

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
    }
    return "unknown status";
}

mesh_status mesh_node_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, size_t* workspace_bytes,
                                      int64_t* cols_capacity) {
    mesh_status st = check_sizes(n_elem, etype, n_vert);
    if (st != MESH_OK) return st;
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    if (n_elem > INT32_MAX / (2 * edges_per_elem(etype))) return MESH_ERR_OVERFLOW;
    NodePlan p;
    if (!plan_node(n_elem, etype, n_vert, &p)) return MESH_ERR_INVALID_ARG;
    *workspace_bytes = p.total;
    *cols_capacity = p.n_pairs;
    return MESH_OK;
}

mesh_status mesh_node_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                int32_t* row_ptr, int32_t* cols, int64_t cols_capacity, void* workspace,
                                size_t workspace_bytes, void* stream) {
    size_t need;
    int64_t cap_hint;
    mesh_status st = mesh_node_neighbors_query(n_elem, etype, n_vert, &need, &cap_hint);
    if (st != MESH_OK) return st;
    if (!row_ptr || !workspace || (n_elem > 0 && !conn) || cols_capacity < 0) return MESH_ERR_INVALID_ARG;
    if (cols_capacity > 0 && !cols) return MESH_ERR_INVALID_ARG;
    if (workspace_bytes < need || !aligned(workspace)) return MESH_ERR_WORKSPACE;
    NodePlan p;
    plan_node(n_elem, etype, n_vert, &p);
    hipError_t e = run_node(p, conn, row_ptr, cols, cols_capacity, workspace, (hipStream_t)stream);
    return e == hipSuccess ? MESH_OK : MESH_ERR_HIP;
}

mesh_status mesh_elem_neighbors_query(int64_t n_elem, int32_t etype, int32_t n_vert, size_t* workspace_bytes,
                                      int64_t* cols_capacity) {
    mesh_status st = check_sizes(n_elem, etype, n_vert);
    if (st != MESH_OK) return st;
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    if (n_elem > INT32_MAX / nodes_per_elem(etype)) return MESH_ERR_OVERFLOW;
    ElemPlan p;
    if (!plan_elem(n_elem, etype, n_vert, &p)) return MESH_ERR_INVALID_ARG;
    *workspace_bytes = p.total;
    *cols_capacity = p.n_slots;
    return MESH_OK;
}

mesh_status mesh_elem_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                int32_t* row_ptr, int32_t* cols, int64_t cols_capacity, void* workspace,
                                size_t workspace_bytes, void* stream) {
    size_t need;
    int64_t cap_hint;
    mesh_status st = mesh_elem_neighbors_query(n_elem, etype, n_vert, &need, &cap_hint);
    if (st != MESH_OK) return st;
    if (!row_ptr || !workspace || (n_elem > 0 && !conn) || cols_capacity < 0) return MESH_ERR_INVALID_ARG;
    if (cols_capacity > 0 && !cols) return MESH_ERR_INVALID_ARG;
    if (workspace_bytes < need || !aligned(workspace)) return MESH_ERR_WORKSPACE;
    ElemPlan p;
    plan_elem(n_elem, etype, n_vert, &p);
    hipError_t e = run_elem(p, conn, row_ptr, cols, cols_capacity, workspace, (hipStream_t)stream);
    return e == hipSuccess ? MESH_OK : MESH_ERR_HIP;
}

mesh_status mesh_batch_node_neighbors_query(int32_t n_mesh, int64_t total_pairs, int32_t total_vert,
                                            int32_t max_vert, size_t* workspace_bytes, int64_t* cols_capacity) {
    if (n_mesh < 0 || total_pairs < 0 || total_vert < 0 || max_vert < 0 || max_vert > total_vert)
        return MESH_ERR_INVALID_ARG;
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    if (total_pairs > INT32_MAX) return MESH_ERR_OVERFLOW;
    BatchPlan p;
    if (!plan_batch(total_pairs, batch_hi_bits(total_vert) + batch_node_lo_bits(max_vert), total_vert, total_vert, &p))
        return MESH_ERR_OVERFLOW;
    *workspace_bytes = p.total;
    *cols_capacity = total_pairs;
    return MESH_OK;
}

mesh_status mesh_batch_node_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                      int64_t total_pairs, int32_t total_vert, int32_t max_vert, int32_t* row_ptr,
                                      int32_t* cols, int64_t cols_capacity, void* workspace, size_t workspace_bytes,
                                      void* stream) {
    size_t need;
    int64_t cap_hint;
    mesh_status st = mesh_batch_node_neighbors_query(n_mesh, total_pairs, total_vert, max_vert, &need, &cap_hint);
    if (st != MESH_OK) return st;
    if (!row_ptr || !workspace || (total_pairs > 0 && (!conn || !segs)) || cols_capacity < 0)
        return MESH_ERR_INVALID_ARG;
    if (cols_capacity > 0 && !cols) return MESH_ERR_INVALID_ARG;
    if (workspace_bytes < need || !aligned(workspace)) return MESH_ERR_WORKSPACE;
    const uint32_t lo = batch_node_lo_bits(max_vert);
    BatchPlan p;
    plan_batch(total_pairs, batch_hi_bits(total_vert) + lo, total_vert, total_vert, &p);
    hipError_t e = run_batch_node(p, conn, segs, n_mesh, lo, total_vert, row_ptr, cols, cols_capacity, workspace,
                                  (hipStream_t)stream);
    return e == hipSuccess ? MESH_OK : MESH_ERR_HIP;
}

mesh_status mesh_batch_elem_neighbors_query(int32_t n_mesh, int64_t total_slots, int32_t total_vert,
                                            size_t* workspace_bytes, int64_t* cols_capacity) {
    if (n_mesh < 0 || total_slots < 0 || total_vert < 0) return MESH_ERR_INVALID_ARG;
    if (!workspace_bytes || !cols_capacity) return MESH_ERR_INVALID_ARG;
    if (total_slots > INT32_MAX) return MESH_ERR_OVERFLOW;
    BatchPlan p;
    if (!plan_batch(total_slots, batch_hi_bits(total_vert), 0, total_vert, &p)) return MESH_ERR_OVERFLOW;
    *workspace_bytes = p.total;
    *cols_capacity = total_slots;
    return MESH_OK;
}

mesh_status mesh_batch_elem_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                      int64_t total_slots, int32_t total_vert, int32_t* row_ptr, int32_t* cols,
                                      int64_t cols_capacity, void* workspace, size_t workspace_bytes, void* stream) {
    size_t need;
    int64_t cap_hint;
    mesh_status st = mesh_batch_elem_neighbors_query(n_mesh, total_slots, total_vert, &need, &cap_hint);
    if (st != MESH_OK) return st;
    if (!row_ptr || !workspace || (total_slots > 0 && (!conn || !segs)) || cols_capacity < 0)
        return MESH_ERR_INVALID_ARG;
    if (cols_capacity > 0 && !cols) return MESH_ERR_INVALID_ARG;
    if (workspace_bytes < need || !aligned(workspace)) return MESH_ERR_WORKSPACE;
    BatchPlan p;
    plan_batch(total_slots, batch_hi_bits(total_vert), 0, total_vert, &p);
    hipError_t e = run_batch_elem(p, conn, segs, n_mesh, total_vert, row_ptr, cols, cols_capacity, workspace,
                                  (hipStream_t)stream);
    return e == hipSuccess ? MESH_OK : MESH_ERR_HIP;
}

int32_t mesh_radix_shape_count(void) { return N_RADIX_SHAPES; }

mesh_status mesh_radix_shape_info(int32_t shape, int32_t* block, int32_t* items) {
    if (shape < 0 || shape >= N_RADIX_SHAPES || !block || !items) return MESH_ERR_INVALID_ARG;
    *block = RADIX_SHAPES[shape].block;
    *items = RADIX_SHAPES[shape].items;
    return MESH_OK;
}

mesh_status mesh_set_radix_shape(int32_t shape) {
    if (shape < -1 || shape >= N_RADIX_SHAPES) return MESH_ERR_INVALID_ARG;
    g_radix_shape.store(shape < 0 ? DEFAULT_RADIX_SHAPE : shape, std::memory_order_relaxed);
    return MESH_OK;
}

int32_t mesh_get_radix_shape(void) { return g_radix_shape.load(std::memory_order_relaxed); }

mesh_status mesh_set_node_sort(int32_t mode) {
    if (mode != MESH_NODE_SORT_FULL_KEY && mode != MESH_NODE_SORT_VERTEX_ROWS && mode != MESH_NODE_SORT_EDGE_ROWS)
        return MESH_ERR_INVALID_ARG;
    g_node_sort.store(mode, std::memory_order_relaxed);
    return MESH_OK;
}

int32_t mesh_get_node_sort(void) { return g_node_sort.load(std::memory_order_relaxed); }

mesh_status mesh_check(const void* workspace, void* stream) {
    if (!workspace) return MESH_ERR_INVALID_ARG;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MESH_ERR_HIP;
    uint32_t err = 0;
    if (hipMemcpy(&err, workspace, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return MESH_ERR_HIP;
    if (err & ERR_INTERNAL) return MESH_ERR_INTERNAL;
    if (err & ERR_INDEX_RANGE) return MESH_ERR_INDEX_RANGE;
    if (err & ERR_CAPACITY) return MESH_ERR_CAPACITY;
    return MESH_OK;
}

}  // extern "C"
