// Batched neighbor build: many independent meshes, of mixed element types
// and sizes, in one launch sequence.  Each mesh is described by a segment
// record in device memory (mesh_segment); its connectivity holds local ids.
// The keys carry the mesh's global vertex range:
//   node relation:    (vert_off[m] + u) << lo_bits | w,   lo_bits = bits of the largest mesh
//   element relation: (vert_off[m] + v) << 32 | e_local
// so one sort and one CSR pass over all meshes give a global row_ptr over all
// vertices whose per-mesh slice equals the single-mesh result, with cols in
// local ids.  The steps are those of the single-mesh pipelines (Sec. 2.2.1,
// 2.2.2): pair generation, LSD radix passes, unique/CSR.
#include "../../include/mesh_neighbors.h"
#include "common.hpp"
#include "csr.hpp"
#include "elements.hpp"
#include "internal.hpp"
#include "launch.hpp"
#include "radix.hpp"
#include "edges.hpp"
#include "erows.hpp"
#include "rows.hpp"

namespace mnb {

constexpr int BH_BLOCK = 512;
constexpr int BH_COPIES = 8;  // per-lane copies of each histogram counter
constexpr int BH_GRID_MAX = 1024;
constexpr int B_MAX_PASS = 8;
constexpr int TK_BCSR = 15;

constexpr int SEG_LUT_SHIFT = 10;
constexpr int LUT_BLOCK = 256;
constexpr int STAGE_HDR = 8;  // int32 header words before the staged ids

static_assert(sizeof(mesh_segment) == 48, "mesh_segment layout");

// Largest m in [lo, hi] with offset(m) <= i (offsets non-decreasing).
// `FIELD` is the byte offset of the int64 offset inside mesh_segment.
template <int FIELD>
__device__ __forceinline__ int find_segment(const mesh_segment* __restrict__ segs, int lo, int hi, int64_t i) {
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t off = *(const int64_t*)((const char*)(segs + mid) + FIELD);
        if (off <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// lut[t] = segment holding position min(t << SEG_LUT_SHIFT, n - 1), for
// t < n_lut = ((n - 1) >> SEG_LUT_SHIFT) + 2.  Position i then lies in a
// segment between lut[i >> SHIFT] and lut[(i >> SHIFT) + 1], usually the
// first, so the per-key search is short.
template <int FIELD>
static __global__ __launch_bounds__(LUT_BLOCK) void segment_lut_kernel(const mesh_segment* __restrict__ segs,
                                                                      int n_mesh, int64_t n, int32_t* __restrict__ lut,
                                                                      int64_t n_lut) {
    const int64_t t = (int64_t)blockIdx.x * LUT_BLOCK + threadIdx.x;
    if (t >= n_lut) return;
    const int64_t pos = tmin<int64_t>(t << SEG_LUT_SHIFT, n - 1);
    lut[t] = find_segment<FIELD>(segs, 0, n_mesh - 1, pos);
}

template <int FIELD>
__device__ __forceinline__ int lut_segment(const mesh_segment* __restrict__ segs, const int32_t* __restrict__ lut,
                                           int64_t i) {
    const int64_t t = i >> SEG_LUT_SHIFT;
    return find_segment<FIELD>(segs, lut[t], lut[t + 1], i);
}

// Per radix tile (TILE consecutive keys): the mesh all of its keys lie in;
// or, for a tile across at most MAX_TILE_SEGS meshes whose ids and keys are
// contiguous (as the offsets of a packed batch are), those meshes; else
// etype = -1 (the per-key path).  Built once per call so that a tile reads
// one record, not a chain of lookups, before staging its ids.
constexpr int TILE_MULTI = -2;
constexpr int MAX_TILE_SEGS = 8;
constexpr int SEG_WORDS = 8;  // staged record of one mesh of a TILE_MULTI tile
struct TileRec {
    int32_t etype;     // >= 0 one mesh; TILE_MULTI several; -1 per-key path
    int32_t n_vert;
    int32_t vert_off;
    uint32_t e0;       // first element of the tile, local to its (first) mesh
    int32_t cnt;       // ids to stage: whole elements from e0 to the tile's last
    int32_t m0;        // TILE_MULTI: first mesh
    int64_t off;       // key offset of the mesh (one mesh)
    int64_t ids;       // index in conn of the first staged id
    int32_t n_seg;     // TILE_MULTI: meshes
    int32_t reserved;
};
static_assert(sizeof(TileRec) == 48, "TileRec layout");

// KIND: 0 element slots, 1 directed pairs, 2 canonical edges (keys of which
// are looked up in the pair table at twice their index).  ids_cap: the most
// ids the source's staging area holds.
template <int KIND>
__device__ __forceinline__ int64_t seg_key_off(const mesh_segment& sg) {
    return KIND == 2 ? sg.pair_off / 2 : KIND == 1 ? sg.pair_off : sg.slot_off;
}
template <int KIND>
__device__ __forceinline__ int seg_keys_per_elem(int32_t et) {
    return KIND == 2 ? edges_per_elem(et) : KIND == 1 ? 2 * edges_per_elem(et) : nodes_per_elem(et);
}

template <int KIND>
static __global__ __launch_bounds__(LUT_BLOCK) void tile_table_kernel(const mesh_segment* __restrict__ segs,
                                                                     const int32_t* __restrict__ lut, int64_t n,
                                                                     int64_t tile, TileRec* __restrict__ recs,
                                                                     int64_t n_tiles, int32_t ids_cap) {
    constexpr int FIELD = KIND ? (int)offsetof(mesh_segment, pair_off) : (int)offsetof(mesh_segment, slot_off);
    constexpr int SCALE = KIND == 2 ? 2 : 1;
    const int64_t t = (int64_t)blockIdx.x * LUT_BLOCK + threadIdx.x;
    if (t >= n_tiles) return;
    const int64_t base = t * tile, last = tmin<int64_t>(base + tile, n) - 1;
    const int m0 = lut_segment<FIELD>(segs, lut, base * SCALE), m1 = lut_segment<FIELD>(segs, lut, last * SCALE);
    TileRec r{};
    r.etype = -1;
    const mesh_segment& sg = segs[m0];
    const int per0 = seg_keys_per_elem<KIND>(sg.etype);
    const int64_t off0 = seg_key_off<KIND>(sg);  // first key of the mesh
    if (per0 == 0 || base < off0 || base >= off0 + per0 * sg.n_elem) {
        recs[t] = r;  // inconsistent records: the per-key path reports them
        return;
    }
    const uint32_t e0 = (uint32_t)((base - off0) / per0);
    if (m0 == m1) {
        if (last < off0 + per0 * sg.n_elem) {
            const uint32_t e1 = (uint32_t)((last - off0) / per0);
            r.etype = sg.etype;
            r.n_vert = sg.n_vert;
            r.vert_off = sg.vert_off;
            r.e0 = e0;
            r.cnt = (int32_t)(e1 - e0 + 1u) * nodes_per_elem(sg.etype);
            r.off = off0;
            r.ids = sg.conn_off + (int64_t)e0 * nodes_per_elem(sg.etype);
        }
    } else if (m1 - m0 < MAX_TILE_SEGS) {
        bool ok = true;
        for (int m = m0; m < m1 && ok; ++m) {
            const mesh_segment& a = segs[m];
            const mesh_segment& b = segs[m + 1];
            const int per = seg_keys_per_elem<KIND>(a.etype);
            ok = (per > 0 || a.n_elem == 0) && seg_key_off<KIND>(a) + per * a.n_elem == seg_key_off<KIND>(b) &&
                 a.conn_off + (int64_t)nodes_per_elem(a.etype) * a.n_elem == b.conn_off;
        }
        const mesh_segment& sl = segs[m1];
        const int per1 = seg_keys_per_elem<KIND>(sl.etype);
        const int64_t off1 = seg_key_off<KIND>(sl);
        ok = ok && per1 > 0 && last >= off1 && last < off1 + per1 * sl.n_elem;
        if (ok) {
            const int64_t ids0 = sg.conn_off + (int64_t)e0 * nodes_per_elem(sg.etype);
            const int64_t ids1 = sl.conn_off + ((last - off1) / per1 + 1) * nodes_per_elem(sl.etype);
            if (ids1 - ids0 <= ids_cap) {
                r.etype = TILE_MULTI;
                r.e0 = e0;
                r.cnt = (int32_t)(ids1 - ids0);
                r.m0 = m0;
                r.n_seg = m1 - m0 + 1;
                r.ids = ids0;
            }
        }
    }
    recs[t] = r;
}

// Stages a TILE_MULTI tile's mesh records (SEG_WORDS words each, after the
// ids area): type, n_vert, vert_off, npe, first id relative to the staged
// ids, key offset (two words).
template <int KIND>
__device__ __forceinline__ void stage_seg_records(const mesh_segment* __restrict__ segs, const TileRec& r,
                                                  int32_t* rec, int tid) {
    if (tid < r.n_seg) {
        const mesh_segment& sg = segs[r.m0 + tid];
        int32_t* q = rec + tid * SEG_WORDS;
        q[0] = sg.etype;
        q[1] = sg.n_vert;
        q[2] = sg.vert_off;
        q[3] = nodes_per_elem(sg.etype);
        q[4] = (int32_t)(sg.conn_off - r.ids);
        const int64_t ko = seg_key_off<KIND>(sg);
        q[6] = (int32_t)ko;
        q[7] = (int32_t)(ko >> 32);
    }
}

// The record of a TILE_MULTI tile's mesh that holds key i (the last one
// whose key offset is at most i; empty meshes share their successor's).
__device__ __forceinline__ const int32_t* find_seg_record(const int32_t* rec, int n_seg, int64_t i) {
    int k = 0;
#pragma unroll
    for (int kk = 1; kk < MAX_TILE_SEGS; ++kk) {
        const int32_t* q = rec + kk * SEG_WORDS;
        const int64_t ko = (int64_t)(((uint64_t)(uint32_t)q[7] << 32) | (uint32_t)q[6]);
        if (kk < n_seg && ko <= i) k = kk;
    }
    return rec + k * SEG_WORDS;
}

// Element, edge nodes and direction of local pair index loc of a mesh of
// type ET (constant divisors).
template <int ET>
__device__ __forceinline__ void pair_of(uint32_t loc, uint32_t* e, int* pa, int* pb, int* dir) {
    constexpr uint32_t KPE = 2 * Elem<ET>::NE;
    *e = loc / KPE;
    const int r = (int)(loc - *e * KPE);
    edge_nodes<ET>(r >> 1, pa, pb);
    *dir = r & 1;
}

// Node key i of the batch: directed edge pair i (the pairs of mesh m start at
// pair_off[m]), or with CANON edge i once (mesh m's edges start at
// pair_off[m] / 2, every pair count being even) as the canonical key
// ((vert_off + min) << lo_bits) | max.
template <bool CANON>
struct BatchNodeKeySrc {
    const int32_t* __restrict__ conn;
    const mesh_segment* __restrict__ segs;
    const int32_t* __restrict__ lut;  // over pair positions
    const TileRec* __restrict__ tiles;  // built for the tile size of the launch
    uint32_t lo_bits;
    int32_t total_vert;
    static constexpr bool kSkipNone = false;
    static constexpr int PAIR_SCALE = CANON ? 2 : 1;  // pair positions per key
    static constexpr int TABLE_KIND = CANON ? 2 : 1;  // tile_table_kernel<KIND>

    template <int ET>
    __device__ __forceinline__ static void locate(uint32_t loc, uint32_t* e, int* pa, int* pb, int* dir) {
        if constexpr (CANON) {
            constexpr uint32_t NE = Elem<ET>::NE;
            *e = loc / NE;
            edge_nodes<ET>((int)(loc - *e * NE), pa, pb);
            *dir = 0;
        } else {
            pair_of<ET>(loc, e, pa, pb, dir);
        }
    }
    __device__ __forceinline__ uint64_t key_of(int32_t x, int32_t y, int dir, int32_t n_vert, int32_t vert_off,
                                               bool* bad) const {
        // the mesh's vertex range must lie inside the batch's
        const bool ok = (uint32_t)x < (uint32_t)n_vert && (uint32_t)y < (uint32_t)n_vert && vert_off >= 0 &&
                        (int64_t)vert_off + n_vert <= (int64_t)total_vert;
        *bad = !ok;
        if (!ok || x == y) return KEY_NONE;
        int32_t u, w;
        if (CANON) {
            u = x < y ? x : y;
            w = x < y ? y : x;
        } else {
            u = dir ? y : x;
            w = dir ? x : y;
        }
        return ((uint64_t)(uint32_t)(vert_off + u) << lo_bits) | (uint64_t)(uint32_t)w;
    }

    // key, or KEY_NONE; *bad is set when an id lies outside the mesh's range
    // or the segment record is inconsistent (unknown type, key beyond it).
    __device__ __forceinline__ uint64_t make(int64_t i, bool* bad) const {
        const int m = lut_segment<offsetof(mesh_segment, pair_off)>(segs, lut, i * PAIR_SCALE);
        const mesh_segment& sg = segs[m];
        const int32_t et = sg.etype;
        const int ne = edges_per_elem(et), npe = nodes_per_elem(et);
        const int64_t loc = i - sg.pair_off / PAIR_SCALE;
        if (ne == 0 || loc < 0 || loc >= 2 * ne / PAIR_SCALE * sg.n_elem) {
            *bad = true;
            return KEY_NONE;
        }
        uint32_t e;
        int pa, pb, dir;
        with_type(et, [&](auto t) { locate<decltype(t)::value>((uint32_t)loc, &e, &pa, &pb, &dir); });
        const int32_t* el = conn + sg.conn_off + (int64_t)e * npe;
        return key_of(el[pa], el[pb], dir, sg.n_vert, sg.vert_off, bad);
    }
    __device__ __forceinline__ uint64_t load(int64_t i) const {
        bool bad;
        return make(i, &bad);
    }

    // ---- staged path: a tile whose keys all lie in one mesh, or in a few
    // contiguous ones, copies their element ids into LDS once (coalesced) and
    // builds its keys there; other tiles use make().  Header words: [0] 1 one
    // mesh, 2 several, 0 not staged; [1] type (one mesh) or mesh count;
    // [2] n_vert, [3] vert_off, [4] first staged element, [6..7] key offset of
    // the mesh.  Several meshes: their records follow the ids area.
    static constexpr bool kStaged = true;
    static constexpr int ids_cap(int tile) { return (CANON ? tile : tile / 2) + 16; }
    template <int TILE>
    static constexpr int stage_words() { return STAGE_HDR + ids_cap(TILE) + MAX_TILE_SEGS * SEG_WORDS; }

    template <int BLOCK, int TILE>
    __device__ __forceinline__ void stage(int64_t tile_base, int64_t n, int32_t* s, int tid) const {
        static_assert(stage_words<TILE>() <= 2 * TILE, "staged ids fit the key staging area");
        constexpr int PER = (ids_cap(TILE) + BLOCK - 1) / BLOCK;
        const TileRec r = tiles[tile_base / TILE];
        if (r.etype == -1) {
            if (tid == 0) s[0] = 0;
            return;
        }
        const int32_t* src = conn + r.ids;  // r.cnt <= ids_cap words
        int32_t* ids = s + STAGE_HDR;
        int32_t v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = q * BLOCK + tid;
            v[q] = i < r.cnt ? src[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = q * BLOCK + tid;
            if (i < r.cnt) ids[i] = v[q];
        }
        if (r.etype == TILE_MULTI) {
            stage_seg_records<TABLE_KIND>(segs, r, ids + ids_cap(TILE), tid);
            if (tid == 0) {
                s[0] = 2;
                s[1] = r.n_seg;
                s[2] = STAGE_HDR + ids_cap(TILE);  // where the records start
            }
        } else if (tid == 0) {
            s[0] = 1;
            s[1] = r.etype;
            s[2] = r.n_vert;
            s[3] = r.vert_off;
            s[4] = (int32_t)r.e0;
            *(int64_t*)(s + 6) = r.off;
        }
    }

    // the tile's header, read once (wave-uniform values); for several meshes
    // etype holds their count and n_vert the word offset of their records
    struct Header {
        int32_t multi, etype, n_vert, vert_off;
        uint32_t e0;
        int64_t off;
    };
    __device__ __forceinline__ bool staged(const int32_t* s) const {
        return __builtin_amdgcn_readfirstlane(s[0]) != 0;
    }
    __device__ __forceinline__ Header header(const int32_t* s) const {
        const int64_t off = *(const int64_t*)(s + 6);
        return {__builtin_amdgcn_readfirstlane(s[0]) == 2, __builtin_amdgcn_readfirstlane(s[1]),
                __builtin_amdgcn_readfirstlane(s[2]), __builtin_amdgcn_readfirstlane(s[3]),
                (uint32_t)__builtin_amdgcn_readfirstlane(s[4]),
                (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(off >> 32)) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)off))};
    }
    // rel: staged position of the mesh's element 0 (negative when the
    // staged ids start past it); element e sits at rel + e * NPE >= 0
    template <int ET>
    __device__ __forceinline__ uint64_t staged_key(const int32_t* ids, int32_t rel, uint32_t loc, int32_t n_vert,
                                                   int32_t vert_off, bool* bad) const {
        uint32_t e;
        int pa, pb, dir;
        locate<ET>(loc, &e, &pa, &pb, &dir);
        const int32_t* el = ids + (rel + (int32_t)e * Elem<ET>::NPE);
        return key_of(el[pa], el[pb], dir, n_vert, vert_off, bad);
    }
    __device__ __forceinline__ uint64_t load_staged(const Header& h, int64_t i, int64_t tile_base, const int32_t* s,
                                                    bool* bad) const {
        const int32_t* ids = s + STAGE_HDR;
        if (h.multi) {
            const int32_t* q = find_seg_record(s + h.n_vert, h.etype, i);
            const uint32_t loc = (uint32_t)(i - (int64_t)(((uint64_t)(uint32_t)q[7] << 32) | (uint32_t)q[6]));
            return with_type(q[0], [&](auto t) {
                return staged_key<decltype(t)::value>(ids, q[4], loc, q[1], q[2], bad);
            });
        }
        const uint32_t loc = (uint32_t)(i - h.off);
        const int32_t e0 = (int32_t)h.e0;  // staged ids start at element e0
        return with_type(h.etype, [&](auto t) {
            constexpr int ET = decltype(t)::value;
            return staged_key<ET>(ids, -Elem<ET>::NPE * e0, loc, h.n_vert, h.vert_off, bad);
        });
    }
    __device__ __forceinline__ uint64_t load_staged(const Header& h, int64_t i, int64_t tile_base,
                                                    const int32_t* s) const {
        bool bad;
        return load_staged(h, i, tile_base, s, &bad);
    }

    // Histogram path: the keys of a tile inside one mesh, whole elements per
    // thread with their ids read once from conn; add(key) for each key whose
    // position lies in [lo, hi).  False if the tile is not inside one mesh.
    template <int ET, int BLOCK, class Add>
    __device__ __forceinline__ void elem_keys(const TileRec& r, int64_t lo, int64_t hi, int tid, Add& add,
                                              bool& bad) const {
        using E = Elem<ET>;
        constexpr int PER = CANON ? E::NE : 2 * E::NE;
        const int n_el = r.cnt / E::NPE;
        const int32_t* ids = conn + r.ids;
#pragma unroll 2
        for (int q = tid; q < n_el; q += BLOCK) {
            int32_t id[E::NPE];
#pragma unroll
            for (int j = 0; j < E::NPE; ++j) id[j] = ids[(int64_t)q * E::NPE + j];
            const int64_t pos0 = r.off + ((int64_t)r.e0 + q) * PER;
#pragma unroll
            for (int k = 0; k < E::NE; ++k) {
#pragma unroll
                for (int dir = 0; dir < (CANON ? 1 : 2); ++dir) {
                    const int64_t pos = pos0 + (CANON ? k : 2 * k + dir);
                    if (pos < lo || pos >= hi) continue;
                    bool b;
                    add(key_of(id[E::A[k]], id[E::B[k]], dir, r.n_vert, r.vert_off, &b));
                    bad |= b;
                }
            }
        }
    }
    template <int BLOCK, int TILE, class Add>
    __device__ __forceinline__ bool hist_tile(int64_t t0, int64_t n, int tid, Add& add, bool& bad) const {
        const TileRec r = tiles[t0 / TILE];
        if (r.etype < 0) return false;
        const int64_t hi = tmin<int64_t>(t0 + TILE, n);
        with_type(r.etype, [&](auto t) { elem_keys<decltype(t)::value, BLOCK>(r, t0, hi, tid, add, bad); });
        return true;
    }
};
using BatchNodePairSrc = BatchNodeKeySrc<false>;
using BatchEdgeSrc = BatchNodeKeySrc<true>;

// (vertex, element) pair of connectivity slot s of the batch.
struct BatchElemPairSrc {
    const int32_t* __restrict__ conn;
    const mesh_segment* __restrict__ segs;
    const int32_t* __restrict__ lut;
    const TileRec* __restrict__ tiles;  // built for the tile size of the launch
    int32_t total_vert;
    static constexpr bool kSkipNone = true;
    // the mesh's vertex range must lie inside the batch's (row_ptr entries
    // are offered at vert_off + v)
    __device__ __forceinline__ bool range_ok(int32_t vert_off, int32_t n_vert) const {
        return vert_off >= 0 && n_vert >= 0 && (int64_t)vert_off + n_vert <= (int64_t)total_vert;
    }
    static constexpr int TABLE_KIND = 0;  // tile_table_kernel<KIND>

    __device__ __forceinline__ uint64_t make(int64_t s, bool* bad) const {
        const int m = lut_segment<offsetof(mesh_segment, slot_off)>(segs, lut, s);
        const mesh_segment& sg = segs[m];
        const int npe = nodes_per_elem(sg.etype);
        const int64_t loc = s - sg.slot_off;
        if (npe == 0 || loc < 0 || loc >= npe * sg.n_elem || !range_ok(sg.vert_off, sg.n_vert)) {
            *bad = true;
            return KEY_NONE;
        }
        const int32_t* el = conn + sg.conn_off;
        const int32_t v = el[loc];
        if ((uint32_t)v >= (uint32_t)sg.n_vert) {
            *bad = true;
            return KEY_NONE;
        }
        *bad = false;
        const uint32_t l32 = (uint32_t)loc;
        const uint32_t e = slot_elem(l32, npe);
        const int j = (int)(l32 - e * (uint32_t)npe);
        const int32_t* first = el + (int64_t)e * npe;
        for (int jj = 0; jj < j; ++jj)
            if (first[jj] == v) return KEY_NONE;  // repeated id inside the element
        return ((uint64_t)(uint32_t)(sg.vert_off + v) << 32) | (uint64_t)e;
    }
    __device__ __forceinline__ uint64_t load(int64_t s) const {
        bool bad;
        return make(s, &bad);
    }

    // staged path as for BatchNodeKeySrc: slot i of a mesh is its conn entry
    // i, so the staged ids are the tile's slots plus the rest of its first
    // and last elements (for the repeat check); header [1] holds npe.
    static constexpr bool kStaged = true;
    static constexpr int ids_cap(int tile) { return tile + 16; }
    template <int TILE>
    static constexpr int stage_words() { return STAGE_HDR + ids_cap(TILE) + MAX_TILE_SEGS * SEG_WORDS; }

    template <int BLOCK, int TILE>
    __device__ __forceinline__ void stage(int64_t tile_base, int64_t n, int32_t* st, int tid) const {
        static_assert(stage_words<TILE>() <= 2 * TILE, "staged ids fit the key staging area");
        constexpr int PER = (ids_cap(TILE) + BLOCK - 1) / BLOCK;
        const TileRec r = tiles[tile_base / TILE];
        if (r.etype == -1) {
            if (tid == 0) st[0] = 0;
            return;
        }
        const int32_t* src = conn + r.ids;  // r.cnt <= ids_cap words
        int32_t* ids = st + STAGE_HDR;
        int32_t v[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = q * BLOCK + tid;
            v[q] = i < r.cnt ? src[i] : 0;
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = q * BLOCK + tid;
            if (i < r.cnt) ids[i] = v[q];
        }
        if (r.etype == TILE_MULTI) {
            stage_seg_records<TABLE_KIND>(segs, r, ids + ids_cap(TILE), tid);
            if (tid == 0) {
                st[0] = 2;
                st[1] = r.n_seg;
                st[2] = STAGE_HDR + ids_cap(TILE);  // where the records start
            }
        } else if (tid == 0) {
            st[0] = 1;
            st[1] = nodes_per_elem(r.etype);
            st[2] = r.n_vert;
            st[3] = r.vert_off;
            st[4] = (int32_t)r.e0;
            *(int64_t*)(st + 6) = r.off;
        }
    }

    // for several meshes, npe holds their count and n_vert the word offset
    // of their records
    struct Header {
        int32_t multi, npe, n_vert, vert_off;
        uint32_t e0;
        int64_t off;
    };
    __device__ __forceinline__ bool staged(const int32_t* st) const {
        return __builtin_amdgcn_readfirstlane(st[0]) != 0;
    }
    __device__ __forceinline__ Header header(const int32_t* st) const {
        const int64_t off = *(const int64_t*)(st + 6);
        return {__builtin_amdgcn_readfirstlane(st[0]) == 2, __builtin_amdgcn_readfirstlane(st[1]),
                __builtin_amdgcn_readfirstlane(st[2]), __builtin_amdgcn_readfirstlane(st[3]),
                (uint32_t)__builtin_amdgcn_readfirstlane(st[4]),
                (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(off >> 32)) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)off))};
    }
    // key of local slot loc of a mesh whose element 0 is staged at rel
    // (negative when the staged ids start past it)
    __device__ __forceinline__ uint64_t staged_key(const int32_t* ids, int32_t rel, int npe, uint32_t loc,
                                                   int32_t n_vert, int32_t vert_off, bool* bad) const {
        const uint32_t e = slot_elem(loc, npe);
        const int j = (int)(loc - e * (uint32_t)npe);
        const int32_t* el = ids + (rel + (int32_t)e * npe);
        const int32_t v = el[j];
        if ((uint32_t)v >= (uint32_t)n_vert || !range_ok(vert_off, n_vert)) {
            *bad = true;
            return KEY_NONE;
        }
        *bad = false;
        // a repeated id inside the element counts once: compare with the
        // element's earlier ids (all reads issued together, up to seven)
        bool first = true;
#pragma unroll
        for (int jj = 0; jj < 7; ++jj) {
            const int32_t w = el[jj < j ? jj : 0];
            first &= jj >= j || w != v;
        }
        return first ? ((uint64_t)(uint32_t)(vert_off + v) << 32) | (uint64_t)e : KEY_NONE;
    }
    __device__ __forceinline__ uint64_t load_staged(const Header& h, int64_t s, int64_t tile_base, const int32_t* st,
                                                    bool* bad) const {
        const int32_t* ids = st + STAGE_HDR;
        if (h.multi) {
            const int32_t* q = find_seg_record(st + h.n_vert, h.npe, s);
            const uint32_t loc = (uint32_t)(s - (int64_t)(((uint64_t)(uint32_t)q[7] << 32) | (uint32_t)q[6]));
            return staged_key(ids, q[4], q[3], loc, q[1], q[2], bad);
        }
        return staged_key(ids, -h.npe * (int32_t)h.e0, h.npe, (uint32_t)(s - h.off), h.n_vert, h.vert_off, bad);
    }
    __device__ __forceinline__ uint64_t load_staged(const Header& h, int64_t s, int64_t tile_base,
                                                    const int32_t* st) const {
        bool bad;
        return load_staged(h, s, tile_base, st, &bad);
    }

    // Histogram path as for BatchNodeKeySrc: slots of whole elements per
    // thread, a repeated id inside an element counted once.
    template <int NPE, int BLOCK, class Add>
    __device__ __forceinline__ void elem_keys(const TileRec& r, int64_t lo, int64_t hi, int tid, Add& add,
                                              bool& bad) const {
        const int n_el = r.cnt / NPE;
        const int32_t* ids = conn + r.ids;
#pragma unroll 2
        for (int q = tid; q < n_el; q += BLOCK) {
            int32_t id[NPE];
#pragma unroll
            for (int j = 0; j < NPE; ++j) id[j] = ids[(int64_t)q * NPE + j];
            const uint32_t e = r.e0 + (uint32_t)q;
            const int64_t pos0 = r.off + (int64_t)e * NPE;
#pragma unroll
            for (int j = 0; j < NPE; ++j) {
                const int64_t pos = pos0 + j;
                if (pos < lo || pos >= hi) continue;
                const int32_t v = id[j];
                if ((uint32_t)v >= (uint32_t)r.n_vert || !range_ok(r.vert_off, r.n_vert)) {
                    bad = true;
                    continue;
                }
                bool first = true;
#pragma unroll
                for (int jj = 0; jj < NPE - 1; ++jj)
                    if (jj < j) first &= id[jj] != v;
                if (first) add(((uint64_t)(uint32_t)(r.vert_off + v) << 32) | (uint64_t)e);
            }
        }
    }
    template <int BLOCK, int TILE, class Add>
    __device__ __forceinline__ bool hist_tile(int64_t t0, int64_t n, int tid, Add& add, bool& bad) const {
        const TileRec r = tiles[t0 / TILE];
        if (r.etype < 0) return false;
        const int64_t hi = tmin<int64_t>(t0 + TILE, n);
        with_type(r.etype, [&](auto t) { elem_keys<Elem<decltype(t)::value>::NPE, BLOCK>(r, t0, hi, tid, add, bad); });
        return true;
    }
};

// Digit histograms (8-bit digits from bit shift0) of the keys a batch source
// generates, the number of participating keys, and the data-error flag.  A
// block takes tiles of BH_BLOCK x ITEMS consecutive keys (the tile size of
// the radix passes, so both use one tile table), staged as in the first pass.
template <class Src, int ITEMS>
__global__ __launch_bounds__(BH_BLOCK) void batch_hist_kernel(Src src, int64_t n, uint32_t shift0, int n_pass,
                                                             uint32_t last_bits, uint32_t copies,
                                                             uint32_t* __restrict__ hist, uint32_t* count,
                                                             uint32_t* err) {
    constexpr int TILE = BH_BLOCK * ITEMS;
    __shared__ __align__(16) int32_t s_stage[Src::template stage_words<TILE>()];  // header holds an int64
    // `copies` (a power of two) copies of every counter, picked by lane: the
    // keys of one small mesh share their high digits, and lanes adding to one
    // address serialise.  Dynamic LDS of n_pass * RADIX * copies words.
    extern __shared__ uint32_t s_hist[];
    __shared__ uint32_t s_keys;
    const int tid = threadIdx.x;
    const uint32_t copy = (uint32_t)tid & (copies - 1);
    if (tid == 0) s_keys = 0;
    for (int i = tid; i < n_pass * RADIX * (int)copies; i += BH_BLOCK) s_hist[i] = 0;
    bool bad_seen = false;
    uint32_t mine = 0;
    auto add = [&](uint64_t k) {
        ++mine;
        for (int p = 0; p < n_pass; ++p) {
            const uint32_t mask = p == n_pass - 1 ? (1u << last_bits) - 1 : RADIX - 1;
            const uint32_t d = p * RADIX + ((uint32_t)(k >> (shift0 + p * RBITS)) & mask);
            atomicAdd(&s_hist[d * copies + copy], 1u);
        }
    };
    __syncthreads();  // counters cleared
    for (int64_t t0 = (int64_t)blockIdx.x * TILE; t0 < n; t0 += (int64_t)gridDim.x * TILE) {
        // a tile inside one mesh: whole elements per thread straight from conn
        if (src.template hist_tile<BH_BLOCK, TILE>(t0, n, tid, add, bad_seen)) continue;
        __syncthreads();  // the previous tile's staged ids are consumed
        src.template stage<BH_BLOCK, TILE>(t0, n, s_stage, tid);
        __syncthreads();
        const bool staged = src.staged(s_stage);
        const auto hdr = src.header(s_stage);  // meaningful only when staged
#pragma unroll 4
        for (int j = 0; j < ITEMS; ++j) {
            const int64_t i = t0 + (int64_t)j * BH_BLOCK + tid;
            if (i >= n) break;
            bool bad = false;
            const uint64_t k = staged ? src.load_staged(hdr, i, t0, s_stage, &bad) : src.make(i, &bad);
            bad_seen |= bad;
            if (Src::kSkipNone && k == KEY_NONE) continue;
            add(k);
        }
    }
    if (bad_seen) set_error(err, ERR_INDEX_RANGE);
    if (mine) atomicAdd(&s_keys, mine);
    __syncthreads();
    if (tid == 0 && s_keys) atomicAdd(count, s_keys);
    for (int i = tid; i < n_pass * RADIX; i += BH_BLOCK) {
        uint32_t v = 0;
        for (uint32_t c = 0; c < copies; ++c) v += s_hist[i * copies + c];
        if (v) atomicAdd(&hist[i], v);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool plan_batch_sort(int64_t n_keys, uint32_t digit_bits, int32_t rows_vert, int32_t total_vert, const Opts& o,
                     BatchPlan* p) {
    if (n_keys < 0 || digit_bits == 0 || digit_bits > 62 || rows_vert < 0 || total_vert < 0) return false;
    *p = BatchPlan{};
    p->opts = o;
    p->n_keys = n_keys;
    p->pp = plan_passes(digit_bits, RBITS);  // batch sorts take 8-bit digits
    if (p->pp.n_pass > B_MAX_PASS) return false;
    p->digit_bits = digit_bits;
    p->n_tiles = ceil_div(n_keys, min_radix_tile());
    p->n_utiles = ceil_div(n_keys, UNIQ_TILE);
    p->rows_vert = rows_vert;
    p->long_cap = rows_vert > 0 ? n_keys / (ROW_SHORT + 1) + 1 : 0;
    const int64_t scan_tiles = rows_vert > 0 ? ceil_div((int64_t)rows_vert + 1, SCAN_TILE) : 0;
    // the rows stages write into the key buffer the sort did not end in, and
    // edge-rows hands the second look-back array to its transposed passes
    const bool two = p->pp.n_pass > 1 || rows_vert > 0;
    size_t off = HEADER_BYTES;
    p->off_hist = off;
    off += align_up(B_MAX_PASS * RADIX * sizeof(uint32_t));
    p->off_hist2 = off;  // edge-rows: histograms of the transposed edges
    off += rows_vert > 0 ? align_up(MAX_KH_PASS * RADIX * sizeof(uint32_t)) : 0;
    p->off_ulb = off;  // CSR look-back, or the rows stage's scan look-back
    off += align_up((size_t)(p->n_utiles > scan_tiles ? p->n_utiles : scan_tiles) * sizeof(uint64_t));
    p->off_lb0 = off;
    off += align_up((size_t)p->n_tiles * RADIX * sizeof(uint64_t));
    p->zero_bytes = off;
    p->off_lb1 = off;
    off += two ? align_up((size_t)p->n_tiles * RADIX * sizeof(uint64_t)) : 0;
    p->off_keys0 = off;
    off += align_up((size_t)n_keys * sizeof(uint64_t));
    p->off_keys1 = off;
    off += two ? align_up((size_t)n_keys * sizeof(uint64_t)) : 0;
    p->off_deg = off;
    off += align_up((size_t)rows_vert * sizeof(int32_t));
    p->off_src = off;
    off += align_up((size_t)rows_vert * sizeof(int64_t));
    p->off_long = off;
    off += align_up((size_t)p->long_cap * sizeof(int64_t));
    p->off_bmin = off;
    off += align_up((size_t)ceil_div((int64_t)total_vert + 1, (int64_t)RF_TILE) * sizeof(int32_t));
    p->off_up = off;
    off += rows_vert > 0 ? align_up(((size_t)rows_vert + 1) * sizeof(int32_t)) : 0;
    p->off_low = off;
    off += rows_vert > 0 ? align_up(((size_t)rows_vert + 1) * sizeof(int32_t)) : 0;
    p->n_lut = n_keys > 0 ? ((n_keys - 1) >> SEG_LUT_SHIFT) + 2 : 0;
    p->off_lut = off;
    off += align_up((size_t)p->n_lut * sizeof(int32_t));
    p->off_tiles = off;  // room for the smallest tile shape
    off += align_up((size_t)p->n_tiles * sizeof(TileRec));
    p->total = off;
    return true;
}

uint32_t batch_node_lo_bits(int32_t max_vert) { return id_bits_for(max_vert); }

bool plan_batch_elem(int64_t total_slots, int32_t total_vert, const Opts& o, BatchPlan* p, size_t) {
    return plan_batch_sort(total_slots, id_bits_for(total_vert), 0, total_vert, o, p);
}

bool plan_batch_node(int64_t total_pairs, int64_t total_slots, int32_t total_vert, int32_t max_vert, const Opts& o,
                     bool internal_elem, BatchNodePlan* p) {
    *p = BatchNodePlan{};
    p->mode = o.node_sort;
    if (p->mode == NS_ELEM_ROWS) {
        if (!plan_batch_elem(total_slots, total_vert, o, &p->bp)) return false;
        size_t off = p->bp.total;
        p->internal_elem = internal_elem;
        if (internal_elem) {
            p->off_erp = off;
            off += align_up(((size_t)total_vert + 1) * sizeof(int32_t));
            p->off_ecols = off;
            off += align_up((size_t)total_slots * sizeof(int32_t));
        }
        off = plan_erows(total_slots, MAX_NPE - 1, total_vert, off, p->bp.off_keys0, p->bp.off_bmin - p->bp.off_keys0,
                         &p->er);
        p->tlist_stride = p->er.n_tiles + 1;
        p->off_tlists = off;
        off += align_up((size_t)ER_LISTS * (size_t)p->tlist_stride * sizeof(int32_t));
        p->total = off;
        return true;
    }
    // full key: the global vertex bits above the local neighbour bits; the
    // rows algorithms: the global vertex bits only, with room for KEY_NONE
    const uint32_t bits = p->mode == NS_FULL_KEY ? id_bits_for(total_vert) + batch_node_lo_bits(max_vert)
                                                 : bits_for_count((int64_t)total_vert + 1);
    if (!plan_batch_sort(total_pairs, bits, p->mode == NS_FULL_KEY ? 0 : total_vert, total_vert, o, &p->bp))
        return false;
    p->total = p->bp.total;
    return true;
}

template <class Src>
static hipError_t batch_pipeline(const BatchPlan& p, Src src, uint32_t shift0, uint32_t csr_lo_bits,
                                 int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap, char* w,
                                 const mesh_segment* segs, int32_t n_mesh, int rows, hipStream_t s) {
    // rows: 0 unique + CSR, 1 vertex-rows stage, 2 edge-rows (src gives
    // canonical edge keys; p.n_keys is the number of edges)
    uint32_t* hdr = (uint32_t*)w;
    uint32_t* err = hdr + HDR_ERR;
    uint32_t* count = hdr + HDR_KEY_COUNT;
    uint32_t* hist = (uint32_t*)(w + p.off_hist);
    uint64_t* ulb = (uint64_t*)(w + p.off_ulb);
    uint64_t* lb[2] = {(uint64_t*)(w + p.off_lb0), (uint64_t*)(w + p.off_lb1)};
    uint64_t* kb[2] = {(uint64_t*)(w + p.off_keys0), (uint64_t*)(w + p.off_keys1)};
    const int shape = p.opts.shape;
    const bool node = !Src::kSkipNone;
    const int n_pass = p.pp.n_pass;

    // the tile size every pass of this call launches with: the tile table,
    // the histogram tiling and the staged id capacity follow it
    const int64_t tile = radix_tile_keys(shape, p.n_keys);
    const int64_t n_tiles = ceil_div(p.n_keys, tile);
    const int grid = (int)tmin<int64_t>(n_tiles, BH_GRID_MAX);
    const uint32_t last_bits = p.pp.width[n_pass - 1];
    const dim3 lut_grid((unsigned)ceil_div(p.n_lut, LUT_BLOCK));
    const int64_t lut_n = rows == 2 ? 2 * p.n_keys : p.n_keys;  // the table is over pair positions
    hipError_t e =
        node ? launch("batch_segment_lut", segment_lut_kernel<offsetof(mesh_segment, pair_off)>, lut_grid,
                      dim3(LUT_BLOCK), s, segs, n_mesh, lut_n, (int32_t*)(w + p.off_lut), p.n_lut)
             : launch("batch_segment_lut", segment_lut_kernel<offsetof(mesh_segment, slot_off)>, lut_grid,
                      dim3(LUT_BLOCK), s, segs, n_mesh, p.n_keys, (int32_t*)(w + p.off_lut), p.n_lut);
    if (e == hipSuccess)
        e = launch("batch_tile_table", tile_table_kernel<Src::TABLE_KIND>,
                   dim3((unsigned)ceil_div(n_tiles, LUT_BLOCK)),
                   dim3(LUT_BLOCK), s, segs, (const int32_t*)(w + p.off_lut), p.n_keys, tile, (TileRec*)(w + p.off_tiles),
                   n_tiles, (int32_t)Src::ids_cap((int)tile));
    const char* hname = node ? "batch_node_hist" : "batch_elem_hist";
    if (e == hipSuccess) {
        const dim3 g(grid), b(BH_BLOCK);
        // at most 32 KB of counters: 8 copies up to 4 passes, 4 beyond
        const uint32_t copies = n_pass <= 4 ? BH_COPIES : BH_COPIES / 2;
        const size_t shm = (size_t)n_pass * RADIX * copies * sizeof(uint32_t);
        if (tile != (int64_t)BH_BLOCK * (tile / BH_BLOCK)) return hipErrorInvalidValue;
        switch (tile / BH_BLOCK) {
            case 12:
                e = launch_shm(hname, batch_hist_kernel<Src, 12>, g, b, shm, s, src, p.n_keys, shift0, n_pass,
                               last_bits, copies, hist, count, err);
                break;
            case 24:
                e = launch_shm(hname, batch_hist_kernel<Src, 24>, g, b, shm, s, src, p.n_keys, shift0, n_pass,
                               last_bits, copies, hist, count, err);
                break;
            case 8:
                e = launch_shm(hname, batch_hist_kernel<Src, 8>, g, b, shm, s, src, p.n_keys, shift0, n_pass,
                               last_bits, copies, hist, count, err);
                break;
            case 16:
                e = launch_shm(hname, batch_hist_kernel<Src, 16>, g, b, shm, s, src, p.n_keys, shift0, n_pass,
                               last_bits, copies, hist, count, err);
                break;
            default: return hipErrorInvalidValue;  // a tile size the table was not built for
        }
    }
    // element relation: the last pass writes cols and offers row starts
    const CsrOut csr{cols, row_ptr, cols ? cols_cap : 0, 32u, 0xffffffffull};  // row_ptr set to INT32_MAX by the caller
    for (int q = 0; q < n_pass && e == hipSuccess; ++q) {
        const uint32_t shift = shift0 + p.pp.shift[q];
        const uint32_t bits = p.pp.width[q];
        uint64_t* out = kb[q & 1];
        uint64_t* lb_next = q + 1 < n_pass || rows == 2 ? lb[(q + 1) & 1] : nullptr;
        const bool last_elem = !node && q + 1 == n_pass;
        if (q == 0 && last_elem)
            e = launch_radix_pass("batch_elem_radix_first", shape, src, csr, p.n_keys, shift, bits, hist, lb[0],
                                  lb_next, hdr + HDR_TICKET0, err, s);
        else if (q == 0)
            e = launch_radix_pass(node ? "batch_node_radix_first" : "batch_elem_radix_first", shape, src, out,
                                  p.n_keys, shift, bits, hist, lb[0], lb_next, hdr + HDR_TICKET0, err, s);
        else if (node)
            e = launch_radix_pass("batch_node_radix", shape, KeyArraySrc{kb[(q - 1) & 1]}, out, p.n_keys, shift,
                                  bits, hist + q * RADIX, lb[q & 1], lb_next, hdr + HDR_TICKET0 + q, err, s);
        else if (last_elem)
            e = launch_radix_pass("batch_elem_radix", shape, CountedKeySrc{kb[(q - 1) & 1], count}, csr, p.n_keys,
                                  shift, bits, hist + q * RADIX, lb[q & 1], lb_next, hdr + HDR_TICKET0 + q, err, s);
        else
            e = launch_radix_pass("batch_elem_radix", shape, CountedKeySrc{kb[(q - 1) & 1], count}, out, p.n_keys,
                                  shift, bits, hist + q * RADIX, lb[q & 1], lb_next, hdr + HDR_TICKET0 + q, err, s);
    }
    if (e != hipSuccess) return e;
    if (!node)
        return launch_rowptr_fill("batch_elem_row_fill", row_ptr, total_vert, count, (int32_t*)(w + p.off_bmin), s);
    if (rows) {
        RowsStage r{kb[(n_pass - 1) & 1], p.n_keys, csr_lo_bits, total_vert, (int32_t*)(w + p.off_deg),
                    (int64_t*)(w + p.off_src), (int32_t*)kb[n_pass & 1], (int64_t*)(w + p.off_long), p.long_cap,
                    hdr + HDR_LONG_COUNT, ulb, hdr + HDR_TICKET0 + TK_BCSR, err};
        if (rows == 1) return launch_rows_stage(true, r, row_ptr, cols, cols_cap, s);
        // edge-rows: each vertex's higher neighbours and their scan, then the
        // transposed edges; the key buffers hold 2 x n_keys keys (pairs)
        int32_t* up_ptr = (int32_t*)(w + p.off_up);
        e = launch_rows_dedup(r, up_ptr, s, true);
        if (e != hipSuccess) return e;
        EdgeStage g{up_ptr, r.deg, r.src, r.temp, total_vert, csr_lo_bits, segs, n_mesh, p.n_keys,
                    {kb[(n_pass - 1) & 1], kb[(n_pass - 1) & 1] + p.n_keys}, (int32_t*)kb[n_pass & 1] + p.n_keys,
                    (uint32_t*)(w + p.off_hist2), {lb[0], lb[1]}, n_pass & 1, hdr + HDR_TICKET0 + 8, shape,
                    p.pp, (int32_t*)(w + p.off_low), (int32_t*)(w + p.off_bmin), err};
        return launch_edge_stage(g, row_ptr, cols, cols_cap, s);
    }
    return launch_unique_csr("batch_node_csr", kb[(n_pass - 1) & 1], p.n_keys, (const uint32_t*)nullptr,
                             csr_lo_bits, total_vert, cols, cols_cap, row_ptr, ulb, hdr + HDR_TICKET0 + TK_BCSR, err,
                             s);
}

hipError_t run_batch_elem(const BatchPlan& p, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                          int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap, void* ws,
                          hipStream_t s, bool keep_err, const FillRegion* extra) {
    const bool empty = p.n_keys == 0 || n_mesh == 0;
    FillRegion fill[3] = {header_fill(ws, p.zero_bytes, keep_err),
                          {row_ptr, (int64_t)total_vert + 1, empty ? 0u : (uint32_t)INT32_MAX}};
    int n_fill = 2;
    if (extra) fill[n_fill++] = *extra;
    hipError_t e = fill_regions(fill, n_fill, s);
    if (e != hipSuccess || empty) return e;
    const int32_t* lut = (const int32_t*)((char*)ws + p.off_lut);
    const TileRec* tiles = (const TileRec*)((char*)ws + p.off_tiles);
    return batch_pipeline(p, BatchElemPairSrc{conn, segs, lut, tiles, total_vert}, 32u, 32u, total_vert, row_ptr,
                          cols, cols_cap, (char*)ws, segs, n_mesh, 0, s);
}

hipError_t run_batch_node(const BatchNodePlan& bn, const int32_t* conn, const mesh_segment* segs, int32_t n_mesh,
                          uint32_t lo_bits, int32_t total_vert, int32_t* row_ptr, int32_t* cols, int64_t cols_cap,
                          void* ws, hipStream_t s, bool keep_err, const int32_t* elem_row_ptr,
                          const int32_t* elem_cols, int64_t elem_cap) {
    const BatchPlan& p = bn.bp;
    const int mode = bn.mode;
    char* w = (char*)ws;
    if (mode == NS_ELEM_ROWS) {
        int32_t* erp = bn.internal_elem ? (int32_t*)(w + bn.off_erp) : const_cast<int32_t*>(elem_row_ptr);
        int32_t* ecols = bn.internal_elem ? (int32_t*)(w + bn.off_ecols) : const_cast<int32_t*>(elem_cols);
        const int64_t ecap = bn.internal_elem ? p.n_keys : elem_cap;
        const FillRegion extra{w + bn.er.off_lb, bn.er.lb_words, 0u};
        hipError_t e = run_batch_elem(p, conn, segs, n_mesh, total_vert, erp, ecols, ecap, ws, s, keep_err, &extra);
        if (e != hipSuccess) return e;
        if (p.n_keys == 0 || n_mesh == 0) return fill_i32(row_ptr, (int64_t)total_vert + 1, 0, s);
        uint32_t* hdr = (uint32_t*)w;
        const ErowsBufs b = erows_bufs(bn.er, w, hdr + HDR_ERR, hdr + HDR_TICKET0 + TK_EROWS);
        static_assert(HDR_TILE_LISTS + ER_LISTS <= (int)(HEADER_BYTES / 4), "tile-list counts inside the header");
        return launch_erows_batch("batch_node", conn, segs, n_mesh, erp, ecols, ecap, total_vert, p.n_keys, row_ptr,
                                  cols, cols_cap, b, (int32_t*)(w + bn.off_tlists), bn.tlist_stride,
                                  hdr + HDR_TILE_LISTS, s);
    }
    const bool empty = p.n_keys == 0 || n_mesh == 0;
    FillRegion fill[3] = {header_fill(ws, p.zero_bytes, keep_err)};
    int n_fill = 1;
    if (!empty && mode != NS_FULL_KEY) fill[n_fill++] = {w + p.off_deg, total_vert, 0u};
    if (!empty && mode == NS_EDGE_ROWS) fill[n_fill++] = {w + p.off_low, (int64_t)total_vert + 1, (uint32_t)INT32_MAX};
    hipError_t e = fill_regions(fill, n_fill, s);
    if (e != hipSuccess) return e;
    if (empty) return fill_i32(row_ptr, (int64_t)total_vert + 1, 0, s);
    const int32_t* lut = (const int32_t*)(w + p.off_lut);
    const TileRec* tiles = (const TileRec*)(w + p.off_tiles);
    if (mode == NS_VERTEX_ROWS)
        return batch_pipeline(p, BatchNodePairSrc{conn, segs, lut, tiles, lo_bits, total_vert}, lo_bits, lo_bits,
                              total_vert, row_ptr, cols, cols_cap, w, segs, n_mesh, 1, s);
    if (mode == NS_EDGE_ROWS) {
        BatchPlan q = p;
        q.n_keys = p.n_keys / 2;  // one canonical key per edge (the plan is sized for the pairs)
        return batch_pipeline(q, BatchEdgeSrc{conn, segs, lut, tiles, lo_bits, total_vert}, lo_bits, lo_bits,
                              total_vert, row_ptr, cols, cols_cap, w, segs, n_mesh, 2, s);
    }
    return batch_pipeline(p, BatchNodePairSrc{conn, segs, lut, tiles, lo_bits, total_vert}, 0u, lo_bits, total_vert,
                          row_ptr, cols, cols_cap, w, segs, n_mesh, 0, s);
}

}  // namespace mnb
