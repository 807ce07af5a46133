// Host side of the ELEM_ROWS node algorithm for meshes of one element type:
// sizing of its stage and the launch with the type's element access
// (erows.hpp).
#include "erows.hpp"
#include "internal.hpp"

namespace mnb {

size_t plan_erows(int64_t n_entries, int slots, int32_t n_vert, size_t off, size_t alias_off, size_t alias_bytes,
                  ErowsPlan* p) {
    p->n_entries = n_entries;
    p->slots = slots;
    p->n_tiles = erows_tiles_bound(n_entries);
    p->long_cap = erows_long_cap(n_entries);
    p->off_lb = off;
    p->lb_words = erows_scan_tiles(n_vert) * 2;
    off += align_up((size_t)p->lb_words * sizeof(uint32_t));
    p->off_tf = off;
    off += align_up(((size_t)p->n_tiles + 1) * sizeof(int32_t));
    p->off_tc = off;
    off += align_up(((size_t)p->n_tiles + 1) * sizeof(int32_t));
    p->off_list = off;
    off += align_up((size_t)p->long_cap * sizeof(int32_t));
    p->off_deg = off;
    off += align_up(((size_t)n_vert + 1) * sizeof(int32_t));
    p->off_soff = off;
    off += align_up(((size_t)n_vert + 1) * sizeof(int16_t));
    p->temp_bytes = (size_t)slots * (size_t)n_entries * sizeof(int32_t);
    if (p->temp_bytes <= alias_bytes) {
        p->off_temp = alias_off;  // dead by the time the stage runs
    } else {
        p->off_temp = off;
        off += align_up(p->temp_bytes);
    }
    return off;
}

ErowsBufs erows_bufs(const ErowsPlan& er, char* ws, uint32_t* err, uint32_t* ticket) {
    uint32_t* hdr = (uint32_t*)ws;
    return ErowsBufs{(int32_t*)(ws + er.off_tf),   (int32_t*)(ws + er.off_tc),   (int32_t*)(ws + er.off_list),
                     er.long_cap,
                     hdr + HDR_LONG_COUNT,          (int32_t*)(ws + er.off_deg),  (int16_t*)(ws + er.off_soff),
                     (int32_t*)(ws + er.off_temp),  (uint64_t*)(ws + er.off_lb),  ticket,
                     err};
}

hipError_t run_erows_uniform(int32_t etype, const ErowsPlan& er, const int32_t* conn, int64_t n_elem,
                             int32_t n_vert, const int32_t* erp, const int32_t* ecols, int64_t ecap,
                             int32_t* row_ptr, int32_t* cols, int64_t cols_cap, char* ws, uint32_t* err,
                             uint32_t* ticket, hipStream_t s) {
    const ErowsBufs b = erows_bufs(er, ws, err, ticket);
    return with_type(etype, [&](auto et) {
        constexpr int ET = decltype(et)::value;
        return launch_erows("node", UniformRows<ET>{conn, n_elem, n_vert}, erp, ecols, ecap, n_vert, er.n_entries,
                            row_ptr, cols, cols_cap, b, s);
    });
}

}  // namespace mnb
