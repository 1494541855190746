// Batching: many small grids in one pipeline run. The grids are placed in
// one "super grid" as disjoint boxes separated by separator planes: vertices
// that belong to no grid, filled with +inf and keyed above every float by the
// order kernel (key 0xFFFFFFFF from the owner map; +inf itself keys lower).
//
// Why the pairs are unchanged: in the lower-star filtration the separator
// vertices (ordered among themselves by index) enter after every real vertex,
// +inf ones included, and a real vertex's lower star holds only vertices of
// its own box. Up to the last real vertex the filtration is the disjoint
// union of the grids' filtrations, so every pair whose birth and death are
// real is a pair of its grid, with the same simplices (the id scheme and the
// Freudenthal split are translation invariant, and the order of equal values
// by index is preserved inside a box). Around each box, the separator region
// is connected and older than every real maximum: it plays the role of the
// virtual maximum that closes the domain boundary in D2 (Sec. 5.2). A grid's
// one infinite D0 class dies in the separator region; it is reported as
// infinite.
#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "dms_internal.h"

namespace dms {

namespace {

constexpr int KB = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + KB - 1) / KB); }

// one wave per row of an item: row r of the batch -> item by binary search
__global__ void k_pack_rows(const float* __restrict__ fields, const BatchSlot* __restrict__ slots, int nslots,
                            int64_t nrows, int64_t X, int64_t XY, float* __restrict__ super, uint32_t* __restrict__ owner) {
    const int64_t row = (int64_t)blockIdx.x * (KB / 64) + (threadIdx.x >> 6);
    if (row >= nrows) return;
    int lo = 0, hi = nslots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slots[mid].row0 <= row) lo = mid;
        else hi = mid - 1;
    }
    const BatchSlot s = slots[lo];
    const int64_t r = row - s.row0;
    const int64_t y = r % s.ny, z = r / s.ny;
    const float* src = fields + s.src_off + (int64_t)s.nx * r;
    const int64_t base = s.ox + X * (s.oy + y) + XY * (s.oz + z);
    for (int x = threadIdx.x & 63; x < s.nx; x += 64) {
        super[base + x] = src[x];
        owner[base + x] = (uint32_t)lo;
    }
}

// max-corner step mask of a simplex type
__device__ inline int corner_mask(int dim, int t) {
    if (dim == 0) return 0;
    if (dim == 1) return t + 1;
    if (dim == 2) return tri_step(t, 0) | tri_step(t, 1);
    return 7;
}

// the item holding all vertices of simplex id (dim) of the super grid, and its
// local id there; -1 if it touches the +inf region
__device__ inline int local_of(const GridDev& g, const uint32_t* owner, const BatchSlot* slots, int dim, int64_t id,
                               int64_t& local) {
    const int64_t a = id / ntypes(dim);
    const int t = (int)(id % ntypes(dim));
    const uint32_t oa = owner[a];
    if (oa == EMPTY32) return -1;
    const int m = corner_mask(dim, t);
    const int64_t far = a + ((m & 1) ? 1 : 0) + ((m & 2) ? g.sy : 0) + ((m & 4) ? g.sz : 0);
    if (far >= g.V || owner[far] != oa) return -1;
    const BatchSlot s = slots[oa];
    const int64_t x = a % g.sy - s.ox, y = (a / g.sy) % g.ny - s.oy, z = a / g.sz - s.oz;
    local = (x + (int64_t)s.nx * (y + (int64_t)s.ny * z)) * ntypes(dim) + t;
    return (int)oa;
}

// Pairs of the super grid -> (item, infinite, local birth) keys and local
// deaths; pairs born in the +inf region get the key ~0 and sort last.
__global__ void k_demux(const dms_pair* __restrict__ pairs, int64_t n, int dim, GridDev g,
                        const uint32_t* __restrict__ owner, const BatchSlot* __restrict__ slots,
                        uint64_t* __restrict__ key, int64_t* __restrict__ death, uint32_t* __restrict__ per_item,
                        uint32_t* kept) {
    const int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    const dms_pair p = pairs[i];
    int64_t lb = 0, ld = -1;
    const int ib = local_of(g, owner, slots, dim, p.birth, lb);
    if (ib < 0) {
        key[i] = ~0ull;
        death[i] = -1;
        return;
    }
    if (p.death >= 0) {
        int64_t l2 = 0;
        const int id = local_of(g, owner, slots, dim + 1, p.death, l2);
        if (id == ib) ld = l2;
    }
    key[i] = ((uint64_t)ib << 33) | ((ld < 0 ? 1ull : 0ull) << 32) | (uint64_t)lb;
    death[i] = ld;
    atomicAdd(&per_item[ib], 1u);
    atomicAdd(kept, 1u);
}

__global__ void k_demux_write(const uint64_t* __restrict__ key, const uint32_t* __restrict__ idx,
                              const int64_t* __restrict__ death, int64_t n, dms_pair* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * KB + threadIdx.x;
    if (i >= n) return;
    out[i].birth = (int64_t)(key[i] & 0xFFFFFFFFull);
    out[i].death = death[idx[i]];
}

}  // namespace

int pack_layers(const int32_t* dims, int n, int X, int Y, int zq, BatchLayout& L, std::string& err) {
    L.slots.assign(n, BatchSlot{});
    std::vector<int> ordr(n);
    std::iota(ordr.begin(), ordr.end(), 0);
    for (int i = 0; i < n; ++i) {
        const int nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
        if (nx < 2 || ny < 2 || nz < 2) {
            err = "every grid side must be >= 2 (item " + std::to_string(i) + ")";
            return -1;
        }
        if (nx + 1 > X || ny + 1 > Y) {
            err = "item " + std::to_string(i) + " is wider than the batch cross-section";
            return -1;
        }
    }
    // tallest first, then widest: layers of boxes, rows ("shelves") inside a layer
    std::stable_sort(ordr.begin(), ordr.end(), [&](int a, int b) {
        if (dims[3 * a + 2] != dims[3 * b + 2]) return dims[3 * a + 2] > dims[3 * b + 2];
        return dims[3 * a + 1] > dims[3 * b + 1];
    });
    int z0 = 0, layer_h = 0, shelf_y = 0, shelf_h = 0, cur_x = 0;
    bool open = false;
    for (int i : ordr) {
        const int fx = dims[3 * i] + 1, fy = dims[3 * i + 1] + 1, fz = dims[3 * i + 2] + 1;
        if (open && cur_x + fx > X) {  // next shelf
            shelf_y += shelf_h;
            shelf_h = 0;
            cur_x = 0;
        }
        if (!open || shelf_y + fy > Y) {  // next layer
            if (open) z0 += layer_h;
            layer_h = fz;
            shelf_y = 0;
            shelf_h = 0;
            cur_x = 0;
            open = true;
        }
        BatchSlot& s = L.slots[i];
        s.nx = dims[3 * i];
        s.ny = dims[3 * i + 1];
        s.nz = dims[3 * i + 2];
        s.ox = cur_x;
        s.oy = shelf_y;
        s.oz = z0;
        cur_x += fx;
        shelf_h = std::max(shelf_h, fy);
    }
    int Z = open ? z0 + layer_h : 2;
    if (zq > 1) Z = (Z + zq - 1) / zq * zq;
    L.X = X;
    L.Y = Y;
    L.Z = std::max(Z, 2);
    int64_t row = 0;
    for (int i = 0; i < n; ++i) {
        L.slots[i].row0 = row;
        row += (int64_t)L.slots[i].ny * L.slots[i].nz;
    }
    L.nrows = row;
    return 0;
}

void launch_pack(const float* fields, const BatchSlot* d_slots, int nslots, int64_t nrows, const BatchLayout& L,
                 float* super, uint32_t* owner, hipStream_t st) {
    const int64_t V = (int64_t)L.X * L.Y * L.Z;
    fill_u32((uint32_t*)super, 0x7F800000u, V, st);  // +inf
    fill_u32(owner, EMPTY32, V, st);
    if (nrows > 0)
        hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)((nrows + KB / 64 - 1) / (KB / 64))), dim3(KB), 0, st, fields,
                           d_slots, nslots, nrows, (int64_t)L.X, (int64_t)L.X * L.Y, super, owner);
}

void launch_demux(const dms_pair* pairs, int64_t n, int dim, const GridDev& g, const uint32_t* owner,
                  const BatchSlot* d_slots, uint64_t* key, int64_t* death, uint32_t* per_item, uint32_t* kept,
                  hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_demux, dim3(nblocks(n)), dim3(KB), 0, st, pairs, n, dim, g, owner, d_slots, key, death,
                           per_item, kept);
}

void launch_demux_write(const uint64_t* key, const uint32_t* idx, const int64_t* death, int64_t n, dms_pair* out,
                        hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_demux_write, dim3(nblocks(n)), dim3(KB), 0, st, key, idx, death, n, out);
}

}  // namespace dms
