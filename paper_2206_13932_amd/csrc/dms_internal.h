// Internal host/device interfaces of the DMS library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/dms.h"
#include "dms_device.h"

namespace dms {

// Critical-cell lists written by the gradient kernel, with packed
// lexicographic keys (bpr = bits per rank):
//   C0 key = rank; C1 key = (r0 << bpr) | r1;
//   C2 key = hi (r0 << bpr) | r1, lo r2; C3 key = hi (r0 << bpr) | r1, lo (r2 << bpr) | r3
// with r0 > r1 > r2 > r3 the vertex ranks in decreasing order.
// Critical cells with their keys in the lexicographic order. A cell's key is
// the rank of its highest vertex x, then the labels (rank order among the
// lower neighbours of x, 4 bits each) of its other vertices, highest first:
// a vertex key has bpr bits, an edge key bpr + 4, a triangle key bpr + 8 and
// a tetrahedron key bpr + 12.
struct CritLists {
    uint32_t* count;  // 4 device counters
    uint32_t cap[4];
    uint32_t* id0;
    uint32_t* key0;
    uint32_t* id1;
    uint64_t* key1;
    uint32_t* id2;
    uint64_t* key2;
    uint32_t* id3;
    uint64_t* key3;
};

constexpr uint32_t EMPTY32 = 0xFFFFFFFFu;
constexpr uint64_t EMPTY64 = ~0ull;

// error flag bits
enum : uint32_t { FLAG_NAN = 1u, FLAG_GUARD = 2u, FLAG_HEAP = 4u, FLAG_WORK = 8u };

// gradient.hip
void launch_gradient(const GridDev& g, const uint32_t* rank, uint8_t* G, int bpr, const CritLists& cl,
                     hipStream_t st);

// sort.hip
void exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t m, uint32_t* part, hipStream_t st);
int64_t scan_part_size(int64_t m);
int64_t sort_tiles(int64_t n);
template <typename K>
int radix_sort_pairs(K* k0, uint32_t* v0, K* k1, uint32_t* v1, int64_t n, int bit_begin, int bit_end,
                     bool implicit_vals, uint32_t* hist, uint32_t* part, hipStream_t st);

// misc.hip
void iota_u32(uint32_t* out, int64_t n, hipStream_t st);
void fill_u32(uint32_t* out, uint32_t v, int64_t n, hipStream_t st);
void fill_u64(uint64_t* out, uint64_t v, int64_t n, hipStream_t st);
// owner: optional map of batched grids (EMPTY32 = separator vertex, keyed above every float)
void float_keys(const float* f, const uint32_t* owner, int64_t n, uint32_t* keys, uint32_t* flags, hipStream_t st);
void rank_scatter(const uint32_t* order, int64_t n, uint32_t* rank, hipStream_t st);
void gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, int64_t n, hipStream_t st);
void gather_u64(const uint64_t* src, const uint32_t* idx, uint64_t* dst, int64_t n, hipStream_t st);
void inverse_perm(const uint32_t* perm, int64_t n, uint32_t* inv, hipStream_t st);  // inv[perm[j]] = j

// pairs.hip -- D0 / D2
// trace_*: c = the critical cells in the gradient kernel's order, pos[i] = the
// position of c[i] in the sorted order (the arcs are written there)
// next: a zeroed u64 work counter
void trace_d0(const GridDev& g, const uint8_t* G, const uint32_t* rank, const uint32_t* c1, const uint32_t* pos,
              int64_t m, uint32_t* na, uint32_t* nb, uint32_t* flags, unsigned long long* next, hipStream_t st);
void tet_positions(const uint32_t* c3_sorted, int64_t m, uint32_t* tet2pos, hipStream_t st);
void trace_d2(const GridDev& g, const uint8_t* G, const uint32_t* tet2pos, const uint32_t* c2, const uint32_t* pos,
              int64_t m, uint32_t* na, uint32_t* nb, uint32_t* flags, unsigned long long* next, hipStream_t st);
// 2D grids (nz = 1): positions of the plane's critical triangles (index
// anchor * 2 + (type == 3), 1 = highest) and the dual tracing of the
// critical edges into triangles, arcs at the edges' decreasing positions
void tri_positions_flat(const uint32_t* c2_sorted, int64_t m, uint32_t* tri2pos, hipStream_t st);
void trace_flat(const GridDev& g, const uint8_t* G, const uint32_t* tri2pos, const uint32_t* c1, const uint32_t* pos,
                int64_t m, uint32_t* na, uint32_t* nb, uint32_t* flags, unsigned long long* next, hipStream_t st);
// jump: one u64 per node, all EMPTY64 (path-halving shortcuts, written by the kernel)
// drop_node0: a column with node 0 (the virtual maximum of the dual
// reductions) is left unpaired, as if the outside were no node; skip_rev
// (optional): column k is left unpaired when skip_rev[m - 1 - k] is set
void reduce_pairs(const uint32_t* na, const uint32_t* nb, int64_t m, uint32_t* owner, uint64_t* bnd,
                  uint64_t* jump, uint32_t* flags, unsigned long long* stats, unsigned long long* next,
                  hipStream_t st, bool drop_node0 = false, const uint8_t* skip_rev = nullptr);
void settled_columns(const uint64_t* bnd, const uint32_t* owner, int64_t m, uint8_t* paired, hipStream_t st);

// batch.hip: one box of the batch layout (origin in the super grid, source
// offset in the caller's packed fields, first row of the box among all rows)
struct BatchSlot {
    int32_t nx, ny, nz;
    int32_t ox, oy, oz;
    int64_t src_off;
    int64_t row0;
};
struct BatchLayout {
    int X = 0, Y = 0, Z = 0;
    int64_t nrows = 0;
    std::vector<BatchSlot> slots;
};
int pack_layers(const int32_t* dims, int n, int X, int Y, int zq, BatchLayout& L, std::string& err);
void launch_pack(const float* fields, const BatchSlot* d_slots, int nslots, int64_t nrows, const BatchLayout& L,
                 float* super, uint32_t* owner, hipStream_t st);
void launch_demux(const dms_pair* pairs, int64_t n, int dim, const GridDev& g, const uint32_t* owner,
                  const BatchSlot* d_slots, uint64_t* key, int64_t* death, uint32_t* per_item, uint32_t* kept,
                  hipStream_t st);
void launch_demux_write(const uint64_t* key, const uint32_t* idx, const int64_t* death, int64_t n, dms_pair* out,
                        hipStream_t st);

// grad.hip
// Allocation-free scatter: scratch in a static device array of
// NOALLOC_SCRATCH_BYTES per GPU, for at most NOALLOC_MAX_CONTRIB
// contributions. noalloc_scratch_init resolves the array's address on the
// current device (call once per device, with it current; 0 = ok);
// scatter_grad_noalloc enqueues the scatter on st and hands back the device
// error flag (-1: device not initialised).
constexpr int64_t NOALLOC_MAX_CONTRIB = (int64_t)1 << 22;
constexpr size_t NOALLOC_SCRATCH_BYTES = ((size_t)65 << 20) + ((size_t)64 << 10);
int noalloc_scratch_init(int device);
int scatter_grad_noalloc(int device, const int64_t* vertex, const float* grad, int64_t n, int64_t nvert, float* out,
                         uint32_t** flag, hipStream_t st);
void scatter_grad(const int64_t* vertex, const float* grad, int64_t n, int64_t nvert, float* out, uint32_t* k0,
                  uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* hist, uint32_t* part, uint32_t* flags,
                  hipStream_t st);

}  // namespace dms
