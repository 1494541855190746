// Device-side definitions shared by the DMS kernels (gfx950).
//
// Implicit Freudenthal/Kuhn triangulation of an nx*ny*nz vertex grid (Sec. 2.1
// of the paper: regular grids are triangulated implicitly, 14-vertex
// neighbourhood in 3D). Vertex id v = x + nx*(y + ny*z). Every simplex is a
// chain w0 < w1 < ... < wk inside one unit cube whose steps are non-empty,
// pairwise disjoint axis sets (3-bit masks: bit0 = x, bit1 = y, bit2 = z).
// Simplex id = anchor * T_k + type with anchor = w0 and T = {1, 7, 12, 6}.
//
// Discrete gradient storage, 26 V bytes: 20 byte planes of V bytes each,
// indexed by the anchor vertex (plane 0 = vertices, 1..7 = edge types, 8..19 =
// triangle types), then one byte per tetrahedron id (anchor * 6 + type): the
// tetrahedra of a cube, which a D2 v-path visits in turn, share a cache line
// (tet_code_at). A byte holds the partner of the simplex:
//   c < 27      partner = cofacet obtained by adding vertex anchor + off27(c),
//               off27(c) = (c%3-1, c/3%3-1, c/9-1)
//   0x80 | i    partner = facet obtained by removing the chain vertex i
//   0xFF        critical simplex
//   0xFE        no such simplex (it would leave the grid)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dms {

constexpr int NSLOT = 74;   // cells of the open star of a vertex: 14 + 36 + 24
constexpr int NNB = 14;     // Freudenthal neighbours
constexpr uint8_t CODE_CRIT = 0xFF;
constexpr uint8_t CODE_NONE = 0xFE;
constexpr int PLANES = 26;  // V bytes each; the last 6 are the tetrahedra by id

// byte of tetrahedron (anchor, type) in the gradient storage
__host__ __device__ constexpr int64_t tet_code_at(int64_t V, int64_t anchor, int type) {
    return 20 * V + anchor * 6 + type;
}

__host__ __device__ constexpr int ntypes(int dim) { return dim == 0 ? 1 : dim == 1 ? 7 : dim == 2 ? 12 : 6; }
__host__ __device__ constexpr int plane_base(int dim) { return dim == 0 ? 0 : dim == 1 ? 1 : dim == 2 ? 8 : 20; }

// Step tables (axis masks) of each simplex type, packed 3 bits per step so
// that a lookup is a shift; per type (s0 | s1 << 4 | s2 << 8):
//   triangles  0x21 0x41 0x61 0x12 0x42 0x52 0x43 0x14 0x24 0x34 0x25 0x16
//   tetrahedra 0x421 0x241 0x412 0x142 0x214 0x124
__host__ __device__ inline int tri_step(int type, int s) {
    const uint64_t lo = 0x714323aa22b1851ull, hi = 0x395ull;  // types 0..9, 10..11: 6 bits each
    const uint64_t w = type < 10 ? lo >> (6 * type) : hi >> (6 * (type - 10));
    return (int)((w >> (3 * s)) & 7);
}
__host__ __device__ inline int tet_step(int type, int s) {
    return (int)((0xa88c314294311ull >> (9 * type + 3 * s)) & 7);  // 9 bits per type
}
__host__ __device__ inline int tri_type(int a, int b) {
    // inverse of tri_step: (A, B) -> type, -1 if not a triangle step pair
    for (int t = 0; t < 12; ++t)
        if (tri_step(t, 0) == a && tri_step(t, 1) == b) return t;
    return -1;
}
// inverse of tet_step for a chain of single-axis steps (a, b, c), a
// permutation of 1, 2, 4: two types per first step, the second of them when
// the second step is the larger of the two left
__host__ __device__ inline int tet_type(int a, int b, int c) {
    return 2 * (a == 1 ? 0 : a == 2 ? 1 : 2) + (b > c ? 1 : 0);
}

struct GridDev {
    int32_t nx, ny, nz;
    int64_t V;
    int64_t sy, sz;  // strides: nx, nx*ny
};

__device__ inline int64_t lin_of_mask(const GridDev& g, int m) {
    return (m & 1 ? 1 : 0) + (m & 2 ? g.sy : 0) + (m & 4 ? g.sz : 0);
}

// vertex ids stay below 2^32 (the library rejects larger grids): 32-bit division
__device__ inline void coords_of(const GridDev& g, int64_t v, int& x, int& y, int& z) {
    const uint32_t u = (uint32_t)v;
    const uint32_t r = u / (uint32_t)g.nx;
    x = (int)(u - r * (uint32_t)g.nx);
    const uint32_t zz = r / (uint32_t)g.ny;
    y = (int)(r - zz * (uint32_t)g.ny);
    z = (int)zz;
}

// Does a chain with total step mask `m` starting at (x, y, z) stay in the grid?
__device__ inline bool fits(const GridDev& g, int x, int y, int z, int m) {
    return (x + (m & 1) < g.nx) && (y + ((m >> 1) & 1) < g.ny) && (z + ((m >> 2) & 1) < g.nz);
}

// off27 code -> linear offset
__device__ inline int64_t lin27(const GridDev& g, int c) {
    int dx = c % 3 - 1, dy = (c / 3) % 3 - 1, dz = c / 9 - 1;
    return dx + dy * g.sy + dz * g.sz;
}

// Monotone 32-bit key of a float: -0 and +0 collapse, NaN flagged by caller.
__device__ inline uint32_t float_key(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7FFFFFFFu) == 0) b = 0;            // -0 -> +0
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ inline bool is_nan_bits(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu) != 0;
}

// a set of slots of the open star: bits 0..63 in lo, slots 64..73 in hi
// (16 bytes, so that one LDS read fetches it)
struct alignas(16) SlotMask {
    uint64_t lo;
    uint32_t hi;
    uint32_t pad;
};

// ---- star tables (computed at compile time, star_tables.h) -----------------
// Neighbour n of x: offset nbv[n] = +mask(n+1) for n < 7, -mask(n-6) else.
// Slot s of the open star: 0..13 edge {x, n}; 14..49 triangle {x, a, b}
// for the 36 link edges; 50..73 tetrahedron {x, a, b, c} for the 24 link
// triangles.
struct StarTables {
    int8_t nbv[NNB][3];
    int8_t l27[NNB];          // nbv.x + 3 nbv.y + 9 nbv.z
    uint16_t lessc[NNB];      // neighbours with a smaller coordinate sum
    uint8_t cpos_pos[NNB];    // 1 if the coordinate sum of n is > 0 (x precedes n)
    uint16_t cellnb[NSLOT];   // neighbour set of each slot
    uint64_t face[NSLOT];     // facets inside the star (slot bitmask, all < 64)
    uint64_t cofc[NSLOT];     // cofacets inside the star (slots 14..73: bit s - 14)
    uint8_t plane[NSLOT];     // gradient byte plane of the slot's simplex
    int8_t aoff[NSLOT][3];    // anchor offset relative to x
    int8_t al27[NSLOT];       // aoff.x + 3 aoff.y + 9 aoff.z
    uint8_t dim[NSLOT];
    uint8_t type[NSLOT];
    SlotMask slnb[16];        // slots whose cell contains neighbour n; rows 14, 15 empty
    uint64_t slnbc[32];       // [2n]: the slots 14..73 of slnb[n] (bit s - 14); 16-byte rows
    // packed for one read when a pair is recorded:
    uint32_t slrec[NSLOT];    // cellnb | (al27 + 13) << 16
    uint32_t nbrec[NNB];      // lessc | cpos_pos << 14 | (l27 + 13) << 16
};

// Persistent work distribution: lanes that are idle take the next work item
// numbers in order. Each wave draws chunks of CHUNK consecutive numbers from
// the global counter *next (one atomic per chunk, not per step: a counter
// hit by every wave at every step serialises the kernel); [pb, pe) is the
// wave's remaining chunk, identical in all its lanes (pass zeros at the
// start). Idle lanes get k; returns false for a lane whose number is past
// total (its work is exhausted). Every active lane of the wave must call it.
template <int64_t CHUNK>
__device__ inline bool wave_take(bool idle, unsigned long long* next, int64_t total, int64_t& k, int64_t& pb,
                                 int64_t& pe) {
    static_assert(CHUNK >= 64, "one refill must serve a whole wave");
    const uint64_t need = __ballot(idle);
    if (need == 0) return true;
    const int lane = threadIdx.x & 63;
    const int64_t cnt = __popcll(need), avail = pe - pb;
    const int64_t r = __popcll(need & ((1ull << lane) - 1));
    if (avail >= cnt) {
        if (idle) k = pb + r;
        pb += cnt;
    } else {
        const int leader = __builtin_ctzll(need);
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(next, (unsigned long long)CHUNK);
        const int64_t nb = (int64_t)__shfl(base, leader, 64);
        if (idle) k = r < avail ? pb + r : nb + (r - avail);
        pb = nb + (cnt - avail);
        pe = nb + CHUNK;
    }
    return !idle || k < total;
}

// Reserve one entry of the list counted by *cnt for every lane that calls
// this with pred set: one atomic per wavefront instead of one per lane (a
// single counter hit by every lane serialises the kernel). The lanes that
// call it together must be converged; lanes that have returned take no part.
__device__ inline uint32_t wave_append(bool pred, uint32_t* cnt) {
    const uint64_t b = __ballot(pred);
    if (b == 0) return 0;
    const int lane = threadIdx.x & 63;
    const int leader = __builtin_ctzll(b);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(b));
    base = __shfl(base, leader, 64);
    return base + (uint32_t)__popcll(b & ((1ull << lane) - 1));
}

// Block-wide list append for kernels over long item ranges. Lane l of the
// block tests items first + it * NT + l (it < ITEMS, reads coalesced); the
// block reserves the places of all its hits with ONE atomicAdd on *cnt, then
// each hit is written by emit. Atomics on one counter from the whole grid
// are executed one after another (about 11 ns each on MI355X), so one per
// wavefront already costs ~3 ms over 17M items; one per NT * ITEMS items
// does not. test(i, payload) -> bool may leave a 64-bit payload for
// emit(i, payload, slot). Every lane of the block must call it (it holds
// two barriers); the order of the hits in the list is unspecified.
template <int NT, int ITEMS, class Test, class Emit>
__device__ inline void block_append(uint32_t* cnt, int64_t first, int64_t n, Test test, Emit emit) {
    static_assert(NT % 64 == 0 && NT <= 1024 && ITEMS <= 32, "block shape");
    __shared__ uint32_t wsum[NT / 64 + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t pay[ITEMS];
    uint32_t hits = 0;  // bit it: item it of this lane is appended
    uint32_t wcount = 0;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t i = first + (int64_t)it * NT + threadIdx.x;
        pay[it] = 0;
        const bool h = i < n && test(i, pay[it]);
        hits |= (uint32_t)h << it;
        wcount += (uint32_t)__popcll(__ballot(h));
    }
    if (lane == 0) wsum[w] = wcount;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int k = 0; k < NT / 64; ++k) {
            const uint32_t c = wsum[k];
            wsum[k] = s;
            s += c;
        }
        wsum[NT / 64] = s ? atomicAdd(cnt, s) : 0u;
    }
    __syncthreads();
    uint32_t at = wsum[NT / 64] + wsum[w];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const bool h = (hits >> it) & 1u;
        const uint64_t b = __ballot(h);
        if (h) emit(first + (int64_t)it * NT + threadIdx.x, pay[it], at + (uint32_t)__popcll(b & ((1ull << lane) - 1)));
        at += (uint32_t)__popcll(b);
    }
}

}  // namespace dms
