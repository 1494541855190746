// Extremum-saddle pairs: D0 (Sec. 5.1) and D2 (Sec. 5.2); on 2D grids the
// maxima's diagram D1 by the same dual tracing one dimension down.
//
// Tracing. D0: each critical edge follows its two descending v-paths (a
// regular vertex continues through its paired edge) to minima. D2: each
// critical triangle follows, on both sides, the dual v-path through
// tetrahedra (a regular tet is left through its paired triangle into the tet
// on the other side) to a maximum or, across the domain boundary, to the
// virtual maximum. Each saddle gives an arc (node_a, node_b); node ids are
// ages: larger id = younger (D0: vertex rank; D2: position in the
// decreasing list of maxima, 0 = virtual maximum, the oldest).
//
// Pairing. Processing the arcs in order with a union-find (younger root
// dies, older root represents) is the reduction of a boundary matrix whose
// columns have two entries (the paper derives the union-find from exactly
// that reduction, Sec. 5.1(c)). It is run lock-free in parallel with the
// compare-and-swap rule of Sec. 7.2: every column reduces independently; it
// claims its pivot (younger node) if free, adds the published boundary of an
// earlier owner, or evicts a later owner and carries on reducing the evicted
// column. Reduced pivots are unique, so the pairs equal the sequential ones.
#include <algorithm>

#include "dms_internal.h"

namespace dms {

namespace {

constexpr int PB = 256;
inline unsigned nblocks(int64_t n) { return (unsigned)((n + PB - 1) / PB); }

constexpr int64_t PATH_GUARD = (int64_t)1 << 22;

// Paths are handed out one at a time (two per critical cell) by wave_take
// (dms_device.h): a lane whose path has ended takes the next one, so the
// lanes of a wave stay busy until the work runs out instead of waiting for
// the wave's longest path; neighbouring cells still go to neighbouring lanes
// (the gradient kernel lists them in grid order), so their v-paths share
// cache lines.
__device__ inline bool take_path(bool idle, unsigned long long* next, int64_t total, int64_t& k, int64_t& pb,
                                 int64_t& pe) {
    return wave_take<256>(idle, next, total, k, pb, pe);
}

// D0: path 2i + s descends from vertex s of critical edge c1[i] to a minimum;
// its rank goes to na (s = 0) or nb (s = 1) at the edge's sorted position.
__global__ __launch_bounds__(PB) void k_trace_d0(GridDev g, const uint8_t* __restrict__ G,
                                                 const uint32_t* __restrict__ rank, const uint32_t* __restrict__ c1,
                                                 const uint32_t* __restrict__ pos, int64_t m,
                                                 uint32_t* __restrict__ na, uint32_t* __restrict__ nb,
                                                 uint32_t* flags, unsigned long long* next) {
    bool have = false;
    int64_t v = 0, steps = 0, k = 0, pb = 0, pe = 0;
    uint32_t* out = nullptr;
    for (;;) {
        if (!take_path(!have, next, 2 * m, k, pb, pe)) break;
        if (!have) {
            const int64_t i = k >> 1;
            const uint32_t e = c1[i];
            v = e / 7;
            if (k & 1) v += lin_of_mask(g, e % 7 + 1);
            out = ((k & 1) ? nb : na) + pos[i];
            steps = 0;
            have = true;
        }
        const uint8_t c = G[v];
        if (c >= 27 || steps >= PATH_GUARD) {  // 0xFF: minimum
            if (c < 27) atomicOr(flags, FLAG_GUARD);
            *out = rank[v];
            have = false;
            continue;
        }
        v += lin27(g, c);
        ++steps;
    }
}

// ---- tetrahedra / triangles in anchor+type form ----------------------------
struct Simp {
    int64_t anchor;
    int type;
};

// The two tetrahedra containing triangle (anchor; A, B), whose anchor has
// coordinates (x, y, z); ok[i] false if outside. out[0] is anchored at
// anchor - lin_of_mask(C) when the triangle spans two steps, else at anchor.
__device__ inline void tri_cofacets_at(const GridDev& g, int64_t anchor, int x, int y, int z, int A, int B,
                                       Simp out[2], bool ok[2]) {
    const int pa = __builtin_popcount(A), pb = __builtin_popcount(B);
    if (pa + pb == 3) {
        if (pa == 2) {
            const int a1 = A & -A, a2 = A ^ a1;
            out[0] = {anchor, tet_type(a1, a2, B)};
            out[1] = {anchor, tet_type(a2, a1, B)};
        } else {
            const int b1 = B & -B, b2 = B ^ b1;
            out[0] = {anchor, tet_type(A, b1, b2)};
            out[1] = {anchor, tet_type(A, b2, b1)};
        }
        ok[0] = ok[1] = true;  // same cube as the triangle
        return;
    }
    const int C = 7 ^ (A | B);
    const int cc[3] = {x, y, z};
    const int ax = C == 1 ? 0 : C == 2 ? 1 : 2;
    ok[0] = cc[ax] > 0;
    out[0] = {anchor - lin_of_mask(g, C), tet_type(C, A, B)};
    ok[1] = fits(g, x, y, z, 7);
    out[1] = {anchor, tet_type(A, B, C)};
}

__device__ inline void tri_cofacets(const GridDev& g, int64_t anchor, int A, int B, Simp out[2], bool ok[2]) {
    int x, y, z;
    coords_of(g, anchor, x, y, z);
    tri_cofacets_at(g, anchor, x, y, z, A, B, out, ok);
}

// Triangle of tet (anchor; s0, s1, s2) opposite chain vertex i.
__device__ inline void tet_facet(const GridDev& g, int64_t anchor, int type, int i, int64_t& ta, int& A, int& B) {
    const int s0 = tet_step(type, 0), s1 = tet_step(type, 1), s2 = tet_step(type, 2);
    ta = anchor;
    if (i == 0) { ta = anchor + lin_of_mask(g, s0); A = s1; B = s2; }
    else if (i == 1) { A = s0 | s1; B = s2; }
    else if (i == 2) { A = s0; B = s1 | s2; }
    else { A = s0; B = s1; }
}

// D2: path 2i + s ascends from side s of critical triangle c2[i] through
// tetrahedra (a regular tet is left through its paired triangle into the tet
// on the other side) to a maximum, whose age goes to na / nb at the
// triangle's position in decreasing order; a path that leaves the domain
// ends at the virtual maximum (age 0).
__global__ __launch_bounds__(PB) void k_trace_d2(GridDev g, const uint8_t* __restrict__ G,
                                                 const uint32_t* __restrict__ tet2pos,
                                                 const uint32_t* __restrict__ c2, const uint32_t* __restrict__ pos,
                                                 int64_t m, uint32_t* __restrict__ na, uint32_t* __restrict__ nb,
                                                 uint32_t* flags, unsigned long long* next) {
    const int64_t V = g.V;
    bool have = false, ok = false;
    int64_t steps = 0, k = 0, pb = 0, pe = 0;
    Simp T{0, 0};
    int tx = 0, ty = 0, tz = 0;  // coordinates of T.anchor, followed step by step
    uint32_t* out = nullptr;
    for (;;) {
        if (!take_path(!have, next, 2 * m, k, pb, pe)) break;
        if (!have) {
            const int64_t i = k >> 1;
            const uint32_t t = c2[i];
            const int type = (int)(t % 12);
            Simp cf[2];
            bool cok[2];
            tri_cofacets(g, t / 12, tri_step(type, 0), tri_step(type, 1), cf, cok);
            const int side = (int)(k & 1);
            T = cf[side];
            ok = cok[side];
            coords_of(g, T.anchor, tx, ty, tz);
            out = (side ? nb : na) + (m - 1 - (int64_t)pos[i]);
            steps = 0;
            have = true;
        }
        if (!ok) {  // virtual maximum
            *out = 0;
            have = false;
            continue;
        }
        if (steps >= PATH_GUARD) {
            atomicOr(flags, FLAG_GUARD);
            *out = 0;
            have = false;
            continue;
        }
        ++steps;
        const uint8_t c = G[tet_code_at(V, T.anchor, T.type)];
        if (c == CODE_CRIT) {
            *out = tet2pos[T.anchor * 6 + T.type];
            have = false;
            continue;
        }
        int64_t ta;
        int A, B;
        tet_facet(g, T.anchor, T.type, c & 3, ta, A, B);
        if (ta != T.anchor) {  // the facet without chain vertex 0 starts one step further
            const int s0 = tet_step(T.type, 0);
            tx += s0 & 1;
            ty += (s0 >> 1) & 1;
            tz += (s0 >> 2) & 1;
        }
        Simp cf[2];
        bool cok[2];
        tri_cofacets_at(g, ta, tx, ty, tz, A, B, cf, cok);
        const bool first_is_T = cf[0].anchor == T.anchor && cf[0].type == T.type;
        const int o = first_is_T ? 1 : 0;
        ok = cok[o];
        if (cf[o].anchor != ta) {  // anchored one step below: anchor - lin_of_mask(C)
            const int C = 7 ^ (A | B);
            tx -= C & 1;
            ty -= (C >> 1) & 1;
            tz -= (C >> 2) & 1;
        }
        T = cf[o];
    }
}

// ---- 2D grids (nz = 1) ---------------------------------------------------
// On a 2D grid the diagram of the maxima is D1, taken from the stable sets
// of the 1-saddles exactly as D2 is in 3D, one dimension down (Sec. 3, 5.2):
// each critical edge follows, on both sides, the dual v-path through
// triangles (a regular triangle is left through its paired edge into the
// triangle on the other side) to a maximum or, across the boundary of the
// square, to the virtual maximum. The plane's triangles are types 0 (steps
// x then y) and 3 (y then x) of the 3D id scheme.

// in-plane cofacet triangles of the edge with anchor a at (x, y) and step mask m
__device__ inline void edge_cofacets_flat(const GridDev& g, int64_t a, int x, int y, int m, Simp cf[2], bool ok[2]) {
    if (m == 1) {  // x edge: type 0 at a (above), type 3 at a - y (below)
        cf[0] = Simp{a, 0};
        ok[0] = y + 1 < g.ny;
        cf[1] = Simp{a - g.sy, 3};
        ok[1] = y > 0;
    } else if (m == 2) {  // y edge: type 3 at a (right), type 0 at a - x (left)
        cf[0] = Simp{a, 3};
        ok[0] = x + 1 < g.nx;
        cf[1] = Simp{a - 1, 0};
        ok[1] = x > 0;
    } else {  // diagonal: the two triangles of the square at a
        cf[0] = Simp{a, 0};
        cf[1] = Simp{a, 3};
        ok[0] = ok[1] = true;
    }
}

// position of a plane triangle in the decreasing list of maxima (1 = highest)
__device__ inline int64_t tri_slot_flat(const Simp& t) { return t.anchor * 2 + (t.type == 3 ? 1 : 0); }

// path 2i + s of critical edge c1[i]: side s to a maximum's position (0 =
// virtual maximum), written at the edge's position in the decreasing order
__global__ __launch_bounds__(PB) void k_trace_flat(GridDev g, const uint8_t* __restrict__ G,
                                                   const uint32_t* __restrict__ tri2pos,
                                                   const uint32_t* __restrict__ c1, const uint32_t* __restrict__ pos,
                                                   int64_t m, uint32_t* __restrict__ na, uint32_t* __restrict__ nb,
                                                   uint32_t* flags, unsigned long long* next) {
    const int64_t V = g.V;
    bool have = false, ok = false;
    int64_t steps = 0, k = 0, pb = 0, pe = 0;
    Simp T{0, 0};
    uint32_t* out = nullptr;
    for (;;) {
        if (!take_path(!have, next, 2 * m, k, pb, pe)) break;
        if (!have) {
            const int64_t i = k >> 1;
            const uint32_t e = c1[i];
            const int64_t a = e / 7;
            int x, y, z;
            coords_of(g, a, x, y, z);
            Simp cf[2];
            bool cok[2];
            edge_cofacets_flat(g, a, x, y, (int)(e % 7) + 1, cf, cok);
            const int side = (int)(k & 1);
            T = cf[side];
            ok = cok[side];
            out = (side ? nb : na) + (m - 1 - (int64_t)pos[i]);
            steps = 0;
            have = true;
        }
        if (!ok) {  // virtual maximum
            *out = 0;
            have = false;
            continue;
        }
        const uint8_t c = G[(int64_t)(8 + T.type) * V + T.anchor];
        if (c == CODE_CRIT) {
            *out = tri2pos[tri_slot_flat(T)];
            have = false;
            continue;
        }
        // a plane triangle can only be paired with one of its edges (0x80 |
        // the chain position of the vertex the edge leaves out)
        if (steps >= PATH_GUARD || (c & 0xFC) != 0x80 || (c & 3) == 3) {
            atomicOr(flags, FLAG_GUARD);
            *out = 0;
            have = false;
            continue;
        }
        ++steps;
        const int p = c & 3;
        const int s0 = T.type == 0 ? 1 : 2, s1 = 3 - s0;  // chain steps: x then y, or y then x
        int64_t ea = T.anchor;
        int em;
        if (p == 0) {  // edge (v1, v2): one step s1 from v1
            ea += lin_of_mask(g, s0);
            em = s1;
        } else if (p == 1) {  // edge (v0, v2): the diagonal
            em = 3;
        } else {  // edge (v0, v1)
            em = s0;
        }
        int x, y, z;
        coords_of(g, ea, x, y, z);
        Simp cf[2];
        bool cok[2];
        edge_cofacets_flat(g, ea, x, y, em, cf, cok);
        const int o = (cf[0].anchor == T.anchor && cf[0].type == T.type) ? 1 : 0;
        ok = cok[o];
        T = cf[o];
    }
}

__global__ void k_tri_positions_flat(const uint32_t* __restrict__ c2, int64_t m, uint32_t* __restrict__ tri2pos) {
    const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (i < m) {
        const uint32_t t = c2[i];
        tri2pos[(int64_t)(t / 12) * 2 + (t % 12 == 3 ? 1 : 0)] = (uint32_t)(m - i);  // highest -> 1
    }
}

__global__ void k_tet_positions(const uint32_t* __restrict__ c3, int64_t m, uint32_t* __restrict__ tet2pos) {
    const int64_t i = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (i < m) tet2pos[c3[i]] = (uint32_t)(m - i);  // highest tet -> 1
}

// ---- lock-free two-entry column reduction ----------------------------------
// Shared state is accessed with relaxed agent-scope atomics: they are coherent
// across the XCDs without cache-wide writeback/invalidate. The only ordering
// needed -- a column's published boundary is complete before its claim -- is
// a wait for the store to complete before the compare-and-swap.
__device__ inline uint32_t ld_rlx(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t ld_rlx64(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_rlx64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Publish order: the data a claim makes visible is written with agent-scope
// atomic stores (sc1, coherent across the XCDs' L2s); vmcnt(0) makes the
// hardware finish them before the claiming atomic is issued, and the two
// signal fences (compiler-only barriers) keep the compiler from moving any
// memory operation across the wait. A release CAS at agent scope would also
// order them, but it adds an L2 writeback (buffer_wbl2) per claim.
__device__ inline void wait_stores() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70); /* vmcnt(0) */
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ inline bool cas32(uint32_t* p, uint32_t expect, uint32_t desired) {
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
}

// Persistent like the tracing kernels: a lane whose column has settled (or
// reduced to zero) takes the next column number from its wave's chunk.
//
// Path halving. Adding any sum of columns to the left of c is a valid step
// for c (it is how the lock-free rule already uses the published, possibly
// unfinished, boundaries of earlier owners); only the reduced pivots are
// unique. So when c goes p0 -> p1 -> p2 through two such sums, {p0, p2} is a
// sum of columns up to the larger of the two highest columns involved, M,
// and jump[p0] = (p2, M) lets any column after M go from p0 to p2 in one
// step: the union-find's path halving, with the column bound that keeps
// each use a left-to-right operation.
__global__ __launch_bounds__(PB) void k_reduce_pairs(const uint32_t* __restrict__ na,
                                                     const uint32_t* __restrict__ nb, int64_t m, uint32_t* owner,
                                                     uint64_t* bnd, uint64_t* jump, uint32_t* flags,
                                                     unsigned long long* stats, unsigned long long* next,
                                                     bool drop_node0, const uint8_t* __restrict__ skip_rev) {
    const int64_t limit = (int64_t)1 << 26;
    unsigned long long steps = 0, evictions = 0;
    bool have = false;
    uint32_t c = 0, p = 0, q = 0;
    uint32_t pp = EMPTY32, pm = 0;  // the pivot before p and the highest column of the sum that led to p
    int64_t k = 0, pb = 0, pe = 0, guard = 0;
    for (;;) {
        if (!take_path(!have, next, m, k, pb, pe)) break;
        if (!have) {
            c = (uint32_t)k;
            p = na[k];
            q = nb[k];
            if (p < q) {
                const uint32_t t = p;
                p = q;
                q = t;
            }
            guard = 0;
            pp = EMPTY32;
            // without the virtual maximum an arc that reaches the outside
            // joins nothing: its column is left unpaired (bnd stays empty) and
            // the lane takes the next one at once
            if ((drop_node0 && q == 0) || (skip_rev && skip_rev[m - 1 - k])) continue;
            have = true;
        }
        if (++guard > limit) {
            atomicOr(flags, FLAG_GUARD);
            have = false;
            continue;
        }
        if (p == q) {  // column reduced to zero: a positive arc
            have = false;
            continue;
        }
        ++steps;
        const uint32_t o = ld_rlx(&owner[p]);
        if (o == EMPTY32) {
            st_rlx64(&bnd[c], ((uint64_t)p << 32) | q);
            wait_stores();
            if (cas32(&owner[p], EMPTY32, c)) have = false;  // settled
            continue;
        }
        if (o < c) {
            uint32_t r, M;
            const uint64_t sc = ld_rlx64(&jump[p]);
            if (sc != EMPTY64 && (uint32_t)sc < c) {  // {p, r}: a sum of columns up to M < c
                r = (uint32_t)(sc >> 32);
                M = (uint32_t)sc;
            } else {
                const uint64_t b = ld_rlx64(&bnd[o]);
                if ((uint32_t)(b >> 32) != p) continue;  // owner moved on; look again
                r = (uint32_t)b;
                M = o;
            }
            if (pp != EMPTY32) st_rlx64(&jump[pp], ((uint64_t)r << 32) | (pm > M ? pm : M));
            // {p, q} + {p, r} = {q, r}
            if (q > r) {
                p = q;
                q = r;
                pp = EMPTY32;
            } else {
                pp = p;
                pm = M;
                p = r;
            }
            continue;
        }
        // o > c: c is earlier and takes the pivot; the evicted column o is
        // carried on by this lane.
        st_rlx64(&bnd[c], ((uint64_t)p << 32) | q);
        wait_stores();
        if (cas32(&owner[p], o, c)) {
            ++evictions;
            const uint64_t b = ld_rlx64(&bnd[o]);
            c = o;
            p = (uint32_t)(b >> 32);
            q = (uint32_t)b;
            pp = EMPTY32;
        }
    }
    if (stats) {  // one atomic per wavefront
        unsigned long long a = steps, b = evictions;
        for (int d = 32; d > 0; d >>= 1) {
            a += __shfl_xor(a, d, 64);
            b += __shfl_xor(b, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&stats[0], a);
            atomicAdd(&stats[1], b);
        }
    }
}

__global__ void k_settled(const uint64_t* __restrict__ bnd, const uint32_t* __restrict__ owner, int64_t m,
                          uint8_t* __restrict__ paired) {
    const int64_t j = (int64_t)blockIdx.x * PB + threadIdx.x;
    if (j >= m) return;
    const uint64_t b = bnd[j];
    paired[j] = (b != EMPTY64 && owner[(uint32_t)(b >> 32)] == (uint32_t)j) ? 1 : 0;
}

}  // namespace

// persistent launches: enough workgroups to fill every CU, fewer for small inputs
inline unsigned trace_blocks(int64_t paths) { return std::min(nblocks(paths), 4096u); }

void trace_d0(const GridDev& g, const uint8_t* G, const uint32_t* rank, const uint32_t* c1, const uint32_t* pos,
              int64_t m, uint32_t* na, uint32_t* nb, uint32_t* flags, unsigned long long* next, hipStream_t st) {
    if (m > 0)
        hipLaunchKernelGGL(k_trace_d0, dim3(trace_blocks(2 * m)), dim3(PB), 0, st, g, G, rank, c1, pos, m, na, nb,
                           flags, next);
}
void tet_positions(const uint32_t* c3_sorted, int64_t m, uint32_t* tet2pos, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_tet_positions, dim3(nblocks(m)), dim3(PB), 0, st, c3_sorted, m, tet2pos);
}
void trace_d2(const GridDev& g, const uint8_t* G, const uint32_t* tet2pos, const uint32_t* c2, const uint32_t* pos,
              int64_t m, uint32_t* na, uint32_t* nb, uint32_t* flags, unsigned long long* next, hipStream_t st) {
    if (m > 0)
        hipLaunchKernelGGL(k_trace_d2, dim3(trace_blocks(2 * m)), dim3(PB), 0, st, g, G, tet2pos, c2, pos, m, na, nb,
                           flags, next);
}
void tri_positions_flat(const uint32_t* c2_sorted, int64_t m, uint32_t* tri2pos, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_tri_positions_flat, dim3(nblocks(m)), dim3(PB), 0, st, c2_sorted, m, tri2pos);
}
void trace_flat(const GridDev& g, const uint8_t* G, const uint32_t* tri2pos, const uint32_t* c1, const uint32_t* pos,
                int64_t m, uint32_t* na, uint32_t* nb, uint32_t* flags, unsigned long long* next, hipStream_t st) {
    if (m > 0)
        hipLaunchKernelGGL(k_trace_flat, dim3(trace_blocks(2 * m)), dim3(PB), 0, st, g, G, tri2pos, c1, pos, m, na,
                           nb, flags, next);
}
void reduce_pairs(const uint32_t* na, const uint32_t* nb, int64_t m, uint32_t* owner, uint64_t* bnd,
                  uint64_t* jump, uint32_t* flags, unsigned long long* stats, unsigned long long* next,
                  hipStream_t st, bool drop_node0, const uint8_t* skip_rev) {
    if (m > 0)
        hipLaunchKernelGGL(k_reduce_pairs, dim3(trace_blocks(m)), dim3(PB), 0, st, na, nb, m, owner, bnd, jump,
                           flags, stats, next, drop_node0, skip_rev);
}
void settled_columns(const uint64_t* bnd, const uint32_t* owner, int64_t m, uint8_t* paired, hipStream_t st) {
    if (m > 0) hipLaunchKernelGGL(k_settled, dim3(nblocks(m)), dim3(PB), 0, st, bnd, owner, m, paired);
}

}  // namespace dms
