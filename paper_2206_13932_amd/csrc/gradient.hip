// Discrete gradient by expansions (ProcessLowerStars, Robins et al.) fused with
// critical-cell extraction -- the paper's Alg. "Zero-persistence skip" and
// Sec. 2.6; parallel over vertices as in Sec. 7.2.
//
// One lane per vertex x. The lower star L(x) holds the cells of the open star
// of x whose other vertices are all lower than x. With the lower neighbours
// relabelled 0..k-1 by rank, a cell of L(x) is the bitmask of its lower
// neighbours, and the lexicographic order of Sec. 2.2 restricted to L(x) is
// the integer order of these masks (the highest differing vertex decides; a
// face is a mask missing only lower bits). Both priority queues are then
// 74-bit slot sets whose minimum is found by comparing 14-bit keys computed
// from the labels, so the simulation is exact and needs no per-lane heap.
//
// A workgroup owns 1024 consecutive vertices and hands them to its lanes in
// order of lower-star size, so that the lanes of a wave, which run the
// simulation in lockstep, have stars of similar size. The partner codes are
// staged in LDS and written out per slot in vertex order (consecutive lanes,
// consecutive bytes): byte stores scattered over the workgroup's span leave
// the L2 as partial lines and multiply the write traffic several times.
//
// Output: gradient byte planes (see dms_device.h) and the critical cells of
// each dimension appended, with their packed lexicographic keys, to per-
// dimension lists (one atomic per wavefront and dimension).
#include "dms_device.h"
#include "dms_internal.h"
#include "star_tables.h"

namespace dms {

namespace {

constexpr int GB = 1024;  // threads per block (vertices handed to lanes by lower-star size)

struct LdsTables {
    uint64_t face[NSLOT];
    uint64_t cof_lo[NSLOT];
    uint16_t cof_hi[NSLOT];
    uint16_t cellnb[NSLOT];
    uint16_t knb[NSLOT];  // the slot's neighbours a | b << 4 | c << 8 (repeated when fewer)
    uint8_t plane[NSLOT];
    int8_t al27[NSLOT];
    int8_t l27[NNB];
    uint16_t lessc[NNB];
    uint8_t cpos_pos[NNB];
    int64_t aofflin[NSLOT];
};

__device__ inline int popc64(uint64_t v) { return __builtin_popcountll(v); }

__device__ inline uint32_t wave_exclusive(uint32_t v, uint32_t& total) {
    const int lane = threadIdx.x & 63;
    uint32_t incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}


__global__ __launch_bounds__(GB) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_gradient(GridDev g, const uint32_t* __restrict__ rank,
                                                 uint8_t* __restrict__ G, int bpr, CritLists cl) {
    __shared__ LdsTables T;
    __shared__ uint8_t scode[NSLOT * GB];  // partner code of each slot, by processing lane
    __shared__ uint32_t bins[NSLOT + 1];   // lanes per lower-star size, then bin offsets
    __shared__ uint16_t perm[GB];          // perm[lane] = the block-local vertex that lane processes
    const int tid = threadIdx.x;
    // cooperative copy of the star tables into LDS
    for (int i = tid; i < NSLOT; i += GB) {
        T.face[i] = kStar.face[i];
        T.cof_lo[i] = kStar.cof_lo[i];
        T.cof_hi[i] = kStar.cof_hi[i];
        T.cellnb[i] = kStar.cellnb[i];
        {
            const uint32_t nb = kStar.cellnb[i], nb2 = nb & (nb - 1), nb3 = nb2 & (nb2 - 1);
            const uint32_t a = __builtin_ctz(nb), b = nb2 ? __builtin_ctz(nb2) : a, c = nb3 ? __builtin_ctz(nb3) : b;
            T.knb[i] = (uint16_t)(a | b << 4 | c << 8);
        }
        T.plane[i] = kStar.plane[i];
        T.al27[i] = kStar.al27[i];
        T.aofflin[i] = (int64_t)kStar.aoff[i][0] + kStar.aoff[i][1] * g.sy + kStar.aoff[i][2] * g.sz;
    }
    for (int i = tid; i < NNB; i += GB) {
        T.l27[i] = kStar.l27[i];
        T.lessc[i] = kStar.lessc[i];
        T.cpos_pos[i] = kStar.cpos_pos[i];
    }
    for (int i = tid; i <= NSLOT; i += GB) bins[i] = 0;
    __syncthreads();

    const int64_t V = g.V;
    // Workgroups are dispatched to the 8 XCDs in turn; XCD k takes the k-th
    // eighth of the grid, in order, so that neighbouring workgroups (which
    // share cache lines of the gradient planes and of the order) meet in one
    // L2. The map is a bijection for any grid size.
    int64_t wg;
    {
        const int64_t n = gridDim.x, q = n / 8, r = n % 8, k = blockIdx.x % 8;
        wg = k * q + (k < r ? k : r) + blockIdx.x / 8;
    }
    const int64_t x0 = wg * GB;

    // lower neighbours of vertex v (bit n: neighbour n exists and is lower);
    // r[n] receives the neighbours' ranks
    auto lower_of = [&](int64_t v, uint32_t& rv, uint32_t (&r)[NNB], int& cx, int& cy, int& cz) {
        coords_of(g, v, cx, cy, cz);
        rv = rank[v];
        uint32_t lower = 0;
#pragma unroll
        for (int n = 0; n < NNB; ++n) {
            const int dx = kStar.nbv[n][0], dy = kStar.nbv[n][1], dz = kStar.nbv[n][2];
            const bool in = (unsigned)(cx + dx) < (unsigned)g.nx && (unsigned)(cy + dy) < (unsigned)g.ny &&
                            (unsigned)(cz + dz) < (unsigned)g.nz;
            // an outside neighbour reads the vertex itself, so that the 14 loads
            // are unconditional and in flight together
            const uint32_t q = rank[in ? v + dx + dy * g.sy + dz * g.sz : v];
            r[n] = in ? q : 0xFFFFFFFFu;
            lower |= ((uint32_t)in & (uint32_t)(q < rv)) << n;  // no branch: no load is sunk into one
        }
        return lower;
    };
    // cells of L(v): the slots whose neighbour sets are lower
    auto cells_of = [&](uint32_t lower, uint64_t& in_lo, uint32_t& in_hi) {
        in_lo = 0;
        in_hi = 0;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const uint32_t nb = kStar.cellnb[s];
            if ((nb & ~lower) == 0) {
                if (s < 64) in_lo |= (uint64_t)1 << s;
                else in_hi |= 1u << (s - 64);
            }
        }
    };

    // ---- 1. own vertex: lower star size, grid-boundary codes, lane assignment ----
    // Lanes of a wave run the lower-star loop in lockstep, so its cost is the
    // largest lower star in the wave. The vertices of the block are handed to
    // lanes in order of lower-star size (a counting sort in LDS), which keeps
    // the stores of each slot inside the block's span.
    const int64_t xo = x0 + tid;
    uint64_t own_lo = 0;
    uint32_t own_hi = 0;
    uint32_t own_lane;  // the lane that processes the own vertex
    {
        uint32_t ncell = 0;
        if (xo < V) {
            uint32_t rv, r[NNB];
            int cx, cy, cz;
            const uint32_t lower = lower_of(xo, rv, r, cx, cy, cz);
            // non-existent simplices anchored at x (upper faces of the grid)
            if (cx == g.nx - 1 || cy == g.ny - 1 || cz == g.nz - 1) {
                for (int t = 0; t < 7; ++t)
                    if (!fits(g, cx, cy, cz, t + 1)) G[(int64_t)(1 + t) * V + xo] = CODE_NONE;
                for (int t = 0; t < 12; ++t)
                    if (!fits(g, cx, cy, cz, tri_step(t, 0) | tri_step(t, 1))) G[(int64_t)(8 + t) * V + xo] = CODE_NONE;
                for (int t = 0; t < 6; ++t) G[tet_code_at(V, xo, t)] = CODE_NONE;
            }
            if (lower) {
                cells_of(lower, own_lo, own_hi);
                ncell = (uint32_t)(popc64(own_lo) + __builtin_popcount(own_hi));
            }
        }
        const uint32_t within = atomicAdd(&bins[ncell], 1u);
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            for (int b = 0; b <= NSLOT; ++b) {
                const uint32_t c = bins[b];
                bins[b] = acc;
                acc += c;
            }
        }
        __syncthreads();
        own_lane = bins[ncell] + within;
        perm[own_lane] = (uint16_t)tid;
        __syncthreads();
    }

#define CODE(s) scode[(s) * GB + tid]

    // ---- 2. the lower star of vertex perm[tid] (ProcessLowerStars) ----
    const int64_t x = x0 + perm[tid];
    const bool active = x < V;
    uint64_t crit_lo = 0;
    uint32_t crit_hi = 0;
    bool crit_vertex = false;
    uint32_t rx = 0;
    uint64_t relpack = 0;  // 4-bit label of each lower neighbour: its rank order among them

    if (active) {
        uint32_t r[NNB];
        int cx, cy, cz;
        const uint32_t lower = lower_of(x, rx, r, cx, cy, cz);
        if (lower == 0) {
            G[x] = CODE_CRIT;  // minimum
            crit_vertex = true;
        } else {
            uint64_t in_lo;
            uint32_t in_hi;
            cells_of(lower, in_lo, in_hi);
            // relabel the lower neighbours by rank: rel[n] = #lower neighbours below n
            int n0 = 0;
#pragma unroll
            for (int n = 0; n < NNB; ++n) {
                uint32_t c = 0;
#pragma unroll
                for (int m = 0; m < NNB; ++m)
                    if (m != n) c += ((lower >> m) & 1) && r[m] < r[n];
                relpack |= (uint64_t)c << (4 * n);
                if (((lower >> n) & 1) && c == 0) n0 = n;
            }
            // key of a cell of L(x): bitmask of its lower neighbours' rank labels
            auto label = [&](uint32_t n) { return (uint32_t)(relpack >> (4 * n)) & 15u; };
            auto key_of = [&](int s) {
                const uint32_t q = T.knb[s];
                return (1u << label(q & 15u)) | (1u << label((q >> 4) & 15u)) | (1u << label(q >> 8));
            };
            auto gput = [&](int s, uint8_t code) { CODE(s) = code; };
            auto unpaired = [&](int s, uint64_t cls_lo) { return popc64(T.face[s] & ~cls_lo); };
            // pair (p, a): p is a facet of a; w = the neighbour of a not in p
            auto pair_cells = [&](int p, int a) {
                const uint32_t w = __builtin_ctz((uint32_t)(T.cellnb[a] & ~T.cellnb[p]));
                const int pos = __builtin_popcount(T.cellnb[a] & T.lessc[w]) + T.cpos_pos[w];
                gput(a, (uint8_t)(0x80 | pos));
                gput(p, (uint8_t)(13 + T.l27[w] - T.al27[p]));
            };
            // x pairs with its lowest edge delta = {x, n0}
            G[x] = (uint8_t)(13 + T.l27[n0]);
            gput(n0, (uint8_t)(0x80 | T.cpos_pos[n0]));
            uint64_t cls_lo = (uint64_t)1 << n0;
            uint32_t cls_hi = 0;
            uint64_t z_lo = (in_lo & 0x3FFFull) & ~cls_lo;  // other edges
            uint32_t z_hi = 0;
            uint64_t o_lo = 0;
            uint32_t o_hi = 0;
            auto push_cofaces = [&](int s) {
                uint64_t c = T.cof_lo[s] & in_lo & ~cls_lo;
                while (c) {
                    const int b = __builtin_ctzll(c);
                    c &= c - 1;
                    if (unpaired(b, cls_lo) == 1) o_lo |= (uint64_t)1 << b;
                }
                uint32_t ch = T.cof_hi[s] & in_hi & ~cls_hi;
                while (ch) {
                    const int b = __builtin_ctz(ch);
                    ch &= ch - 1;
                    if (unpaired(64 + b, cls_lo) == 1) o_hi |= 1u << b;
                }
            };
            auto pop_min = [&](uint64_t& lo, uint32_t& hi) {
                int best = -1;
                uint32_t bk = 0xFFFFFFFFu;
                uint64_t m = lo;
                while (m) {
                    const int s = __builtin_ctzll(m);
                    m &= m - 1;
                    const uint32_t k = key_of(s);
                    if (k < bk) { bk = k; best = s; }
                }
                uint32_t h = hi;
                while (h) {
                    const int s = 64 + __builtin_ctz(h);
                    h &= h - 1;
                    const uint32_t k = key_of(s);
                    if (k < bk) { bk = k; best = s; }
                }
                if (best < 64) lo &= ~((uint64_t)1 << best);
                else hi &= ~(1u << (best - 64));
                return best;
            };
            push_cofaces(n0);
            for (int guard = 0; guard < 4 * NSLOT; ++guard) {
                while (o_lo | o_hi) {
                    const int a = pop_min(o_lo, o_hi);
                    const bool done = a < 64 ? ((cls_lo >> a) & 1) : ((cls_hi >> (a - 64)) & 1);
                    if (done) continue;
                    const uint64_t u = T.face[a] & ~cls_lo;
                    if (u == 0) {
                        if (a < 64) z_lo |= (uint64_t)1 << a;
                        else z_hi |= 1u << (a - 64);
                        continue;
                    }
                    const int p = __builtin_ctzll(u);
                    pair_cells(p, a);
                    cls_lo |= (uint64_t)1 << p;
                    if (a < 64) cls_lo |= (uint64_t)1 << a;
                    else cls_hi |= 1u << (a - 64);
                    z_lo &= ~((uint64_t)1 << p);
                    push_cofaces(a);
                    push_cofaces(p);
                }
                if (!(z_lo | z_hi)) break;
                const int c = pop_min(z_lo, z_hi);
                if (c < 64) { cls_lo |= (uint64_t)1 << c; crit_lo |= (uint64_t)1 << c; }
                else { cls_hi |= 1u << (c - 64); crit_hi |= 1u << (c - 64); }
                gput(c, CODE_CRIT);
                push_cofaces(c);
            }
        }
    }
    __syncthreads();

    // ---- 3. gradient codes of the own vertex's lower star: one store per slot,
    // consecutive lanes -> consecutive bytes ----
    {
        const uint32_t col = own_lane;
        for (int s = 0; s < NSLOT; ++s) {
            const bool w = s < 64 ? ((own_lo >> s) & 1) : ((own_hi >> (s - 64)) & 1);
            if (w) {
                const int pl = T.plane[s];  // the same in every lane
                const int64_t a = xo + T.aofflin[s];
                G[pl < 20 ? (int64_t)pl * V + a : tet_code_at(V, a, pl - 20)] = scode[s * GB + col];
            }
        }
    }

    // ---- critical-cell lists of vertex x (every lane of the block takes part) ----
    // keys in the lexicographic order: the rank of x, then the labels of the
    // other vertices, highest first, 4 bits each (see CritLists)
    auto lab = [&](int n) { return (uint32_t)(relpack >> (4 * n)) & 15u; };
    const uint64_t E_MASK = 0x3FFFull, T_MASK = ((1ull << 50) - 1) & ~0x3FFFull;
    const uint64_t Q_LO = ~((1ull << 50) - 1);
    uint32_t c0 = crit_vertex ? 1 : 0;
    uint32_t c1 = popc64(crit_lo & E_MASK);
    uint32_t c2 = popc64(crit_lo & T_MASK);
    uint32_t c3 = popc64(crit_lo & Q_LO) + __builtin_popcount(crit_hi);
    // places in the four lists: one atomicAdd per list and workgroup (a list
    // counter hit by every wavefront of the grid serialises the kernel at
    // about 11 ns per atomic); bins is free again after the counting sort
    constexpr int NWV = GB / 64;
    static_assert(4 * (NWV + 1) <= NSLOT + 1, "list sums must fit in bins");
    uint32_t base[4];
    {
        const int lane = tid & 63, w = tid >> 6;
        const uint32_t cc[4] = {c0, c1, c2, c3};
        uint32_t ex[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t tot;
            ex[d] = wave_exclusive(cc[d], tot);
            if (lane == 63) bins[d * (NWV + 1) + w] = tot;
        }
        __syncthreads();
        if (tid < 4) {
            uint32_t* b = bins + tid * (NWV + 1);
            uint32_t sum = 0;
            for (int k = 0; k < NWV; ++k) {
                const uint32_t c = b[k];
                b[k] = sum;
                sum += c;
            }
            b[NWV] = sum ? atomicAdd(&cl.count[tid], sum) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int d = 0; d < 4; ++d) base[d] = bins[d * (NWV + 1) + NWV] + bins[d * (NWV + 1) + w] + ex[d];
    }
    {
        uint32_t at = base[0];
        if (c0 && at < cl.cap[0]) { cl.id0[at] = (uint32_t)x; cl.key0[at] = rx; }
    }
    {
        uint32_t at = base[1];
        uint64_t m = crit_lo & E_MASK;
        while (m) {
            const int s = __builtin_ctzll(m);  // edge slot s joins x to neighbour s
            m &= m - 1;
            if (at < cl.cap[1]) {
                const int64_t a = x + T.aofflin[s];
                cl.id1[at] = (uint32_t)(a * 7 + (T.plane[s] - 1));
                cl.key1[at] = ((uint64_t)rx << 4) | lab(s);
            }
            ++at;
        }
    }
    {
        uint32_t at = base[2];
        uint64_t m = crit_lo & T_MASK;
        while (m) {
            const int s = __builtin_ctzll(m);
            m &= m - 1;
            if (at < cl.cap[2]) {
                const int64_t a = x + T.aofflin[s];
                cl.id2[at] = (uint32_t)(a * 12 + (T.plane[s] - 8));
                const uint32_t nb = T.cellnb[s];
                const uint32_t la = lab(__builtin_ctz(nb)), lb = lab(31 - __builtin_clz(nb));
                const uint32_t hi = la > lb ? la : lb, lo = la > lb ? lb : la;
                cl.key2[at] = ((uint64_t)rx << 8) | (hi << 4) | lo;
            }
            ++at;
        }
    }
    {
        uint32_t at = base[3];
        uint64_t m = crit_lo & Q_LO;
        uint32_t h = crit_hi;
        while (m | h) {
            int s;
            if (m) { s = __builtin_ctzll(m); m &= m - 1; }
            else { s = 64 + __builtin_ctz(h); h &= h - 1; }
            if (at < cl.cap[3]) {
                const int64_t a = x + T.aofflin[s];
                cl.id3[at] = (uint32_t)(a * 6 + (T.plane[s] - 20));
                uint32_t nb = T.cellnb[s];
                uint32_t ll[3];
                for (int i = 0; i < 3; ++i) {
                    const int n = __builtin_ctz(nb);
                    nb &= nb - 1;
                    ll[i] = lab(n);
                }
                // sort the three labels descending
                uint32_t t0 = ll[0], t1 = ll[1], t2 = ll[2], t;
                if (t0 < t1) { t = t0; t0 = t1; t1 = t; }
                if (t1 < t2) { t = t1; t1 = t2; t2 = t; }
                if (t0 < t1) { t = t0; t0 = t1; t1 = t; }
                cl.key3[at] = ((uint64_t)rx << 12) | (t0 << 8) | (t1 << 4) | t2;
            }
            ++at;
        }
    }
#undef KEY
#undef CODE
}

}  // namespace

void launch_gradient(const GridDev& g, const uint32_t* rank, uint8_t* G, int bpr, const CritLists& cl,
                     hipStream_t st) {
    const int64_t blocks = (g.V + GB - 1) / GB;
    hipLaunchKernelGGL(k_gradient, dim3((unsigned)blocks), dim3(GB), 0, st, g, rank, G, bpr, cl);
}

}  // namespace dms
