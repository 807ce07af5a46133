// HIP graphs of the pipelines: each capture records the launch sequence of
// one call of an entry point, with its pointers and sizes, on a private
// capturing stream and instantiates it; mesh_graph_launch replays that
// sequence on any stream.  Every step of the pipelines (clears included) is a
// kernel, so a replay recomputes the result from the current contents of the
// captured input buffers, exactly as an eager call on them would.
#include <hip/hip_runtime.h>

#include <new>

#include "../../include/mesh_neighbors.h"

struct mesh_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// A bounded-memory build waits on its stream for a histogram, which a capture
// cannot hold: such options are refused before capturing.
bool chunked(const mesh_options* o) { return o && o->chunk_keys > 0; }

template <typename F>
mesh_status capture(mesh_graph* out, F&& call) {
    if (!out) return MESH_ERR_INVALID_ARG;
    *out = nullptr;
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return MESH_ERR_HIP;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return MESH_ERR_HIP;
    }
    mesh_status st = call((void*)cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st != MESH_OK || e != hipSuccess || !g) {
        if (g) (void)hipGraphDestroy(g);
        return st != MESH_OK ? st : MESH_ERR_HIP;
    }
    hipGraphExec_t x = nullptr;
    if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return MESH_ERR_HIP;
    }
    mesh_graph h = new (std::nothrow) mesh_graph_s;
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return MESH_ERR_HIP;  // host allocation of the handle failed
    }
    h->graph = g;
    h->exec = x;
    *out = h;
    return MESH_OK;
}

}  // namespace

extern "C" {

mesh_status mesh_graph_node_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                      int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                      const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                      mesh_graph* graph) {
    if (chunked(opts)) {
        if (graph) *graph = nullptr;
        return MESH_ERR_INVALID_ARG;
    }
    return capture(graph, [&](void* s) {
        return mesh_node_neighbors(conn, n_elem, etype, n_vert, row_ptr, cols, cols_capacity, opts, workspace,
                                   workspace_bytes, s);
    });
}

mesh_status mesh_graph_elem_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                      int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                      const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                      mesh_graph* graph) {
    if (chunked(opts)) {
        if (graph) *graph = nullptr;
        return MESH_ERR_INVALID_ARG;
    }
    return capture(graph, [&](void* s) {
        return mesh_elem_neighbors(conn, n_elem, etype, n_vert, row_ptr, cols, cols_capacity, opts, workspace,
                                   workspace_bytes, s);
    });
}

mesh_status mesh_graph_neighbors(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                 int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                 int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                 const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                 mesh_graph* graph) {
    if (chunked(opts)) {
        if (graph) *graph = nullptr;
        return MESH_ERR_INVALID_ARG;
    }
    return capture(graph, [&](void* s) {
        return mesh_neighbors(conn, n_elem, etype, n_vert, node_row_ptr, node_cols, node_cols_capacity, elem_row_ptr,
                              elem_cols, elem_cols_capacity, opts, workspace, workspace_bytes, s);
    });
}

mesh_status mesh_graph_batch_node_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                            int64_t total_pairs, int64_t total_slots, int32_t total_vert,
                                            int32_t max_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_capacity,
                                            const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                            mesh_graph* graph) {
    return capture(graph, [&](void* s) {
        return mesh_batch_node_neighbors(conn, segs, n_mesh, total_pairs, total_slots, total_vert, max_vert, row_ptr,
                                         cols, cols_capacity, opts, workspace, workspace_bytes, s);
    });
}

mesh_status mesh_graph_batch_elem_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                            int64_t total_slots, int32_t total_vert, int32_t* row_ptr,
                                            int32_t* cols, int64_t cols_capacity, const mesh_options* opts,
                                            void* workspace, size_t workspace_bytes, mesh_graph* graph) {
    return capture(graph, [&](void* s) {
        return mesh_batch_elem_neighbors(conn, segs, n_mesh, total_slots, total_vert, row_ptr, cols, cols_capacity,
                                         opts, workspace, workspace_bytes, s);
    });
}

mesh_status mesh_graph_batch_neighbors(const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                                       int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert,
                                       int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                       int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                       const mesh_options* opts, void* workspace, size_t workspace_bytes,
                                       mesh_graph* graph) {
    return capture(graph, [&](void* s) {
        return mesh_batch_neighbors(conn, segs, n_mesh, total_pairs, total_slots, total_vert, max_vert, node_row_ptr,
                                    node_cols, node_cols_capacity, elem_row_ptr, elem_cols, elem_cols_capacity, opts,
                                    workspace, workspace_bytes, s);
    });
}

mesh_status mesh_graph_launch(mesh_graph graph, void* stream) {
    if (!graph || !graph->exec) return MESH_ERR_INVALID_ARG;
    return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? MESH_OK : MESH_ERR_HIP;
}

mesh_status mesh_graph_destroy(mesh_graph graph) {
    if (!graph) return MESH_OK;
    hipError_t e1 = graph->exec ? hipGraphExecDestroy(graph->exec) : hipSuccess;
    hipError_t e2 = graph->graph ? hipGraphDestroy(graph->graph) : hipSuccess;
    delete graph;
    return (e1 == hipSuccess && e2 == hipSuccess) ? MESH_OK : MESH_ERR_HIP;
}

}  // extern "C"
