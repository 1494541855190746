// Discrete gradient by expansions (ProcessLowerStars, Robins et al.) fused with
// critical-cell extraction -- the paper's Alg. "Zero-persistence skip" and
// Sec. 2.6; parallel over vertices as in Sec. 7.2.
//
// One lane per vertex x; the per-vertex algorithm is lower_star.h (slot sets
// as priority queues, minimum by elimination over the rank labels of the
// lower neighbours, labels from a sorting network).
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
// dimension lists (one atomic per workgroup and dimension).
#include "dms_device.h"
#include "dms_internal.h"
#include "star_tables.h"
#include "lower_star.h"

namespace dms {

namespace {

constexpr int GB = 1024;  // threads per block (vertices handed to lanes by lower-star size)

struct LdsTables {
    uint64_t face[NSLOT];
    uint64_t cofc[NSLOT];
    uint16_t cellnb[NSLOT];
    SlotMask slnb[16];  // slots holding neighbour n (rows 14, 15 empty)
    uint64_t slnbc[32];  // the same rows for slots 14..73, one word each (16-byte stride)
    uint32_t slrec[NSLOT];
    uint32_t nbrec[NNB];
    uint8_t plane[NSLOT];
    int8_t l27[NNB];
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


// PACKED: ranks below 2^28 (the labels come from one 32-bit sorting network)
template <bool PACKED>
__global__ __launch_bounds__(GB) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_gradient(GridDev g, const uint32_t* __restrict__ rank,
                                                 uint8_t* __restrict__ G, int bpr, CritLists cl) {
    // one block of LDS with the tables first: their addresses stay below 64 KB,
    // so table reads take the base as an instruction offset instead of adds
    struct Shared {
        LdsTables T;
        uint8_t scode[NSLOT * GB];  // partner code of each slot, by processing lane
        uint32_t bins[NSLOT + 1];   // lanes per lower-star size, then bin offsets
        uint16_t perm[GB];          // perm[lane] = the block-local vertex that lane processes
    };
    __shared__ Shared S;
    LdsTables& T = S.T;
    uint8_t* const scode = S.scode;
    uint32_t* const bins = S.bins;
    uint16_t* const perm = S.perm;
    const int tid = threadIdx.x;
    // cooperative copy of the star tables into LDS
    for (int i = tid; i < NSLOT; i += GB) {
        T.face[i] = kStar.face[i];
        T.cofc[i] = kStar.cofc[i];
        T.cellnb[i] = kStar.cellnb[i];
        T.slrec[i] = kStar.slrec[i];
        T.plane[i] = kStar.plane[i];
        T.aofflin[i] = (int64_t)kStar.aoff[i][0] + kStar.aoff[i][1] * g.sy + kStar.aoff[i][2] * g.sz;
    }
    for (int i = tid; i < 16; i += GB) T.slnb[i] = kStar.slnb[i];
    for (int i = tid; i < 32; i += GB) T.slnbc[i] = kStar.slnbc[i];
    for (int i = tid; i < NNB; i += GB) {
        T.nbrec[i] = kStar.nbrec[i];
        T.l27[i] = kStar.l27[i];
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
    // ---- 1. own vertex: lower star size, grid-boundary codes, lane assignment ----
    // Lanes of a wave run the lower-star loop in lockstep, so its cost is the
    // largest lower star in the wave. The vertices of the block are handed to
    // lanes in order of lower-star size (a counting sort in LDS), which keeps
    // the stores of each slot inside the block's span.
    // The labels, the star's cells and the rank found here are handed to the
    // lane that processes the vertex through the code buffer, free until the
    // lower-star loop (words of 1024 lanes: inv0, inv1, rank, lower | in_hi
    // << 16, in_lo low, in_lo high).
    uint32_t* const stash = (uint32_t*)scode;
    static_assert(6 * GB * 4 <= NSLOT * GB, "the hand-over fits the code buffer");
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
            uint32_t inv0 = 0, inv1 = 0;
            // non-existent simplices anchored at x (upper faces of the grid)
            if (cx == g.nx - 1 || cy == g.ny - 1 || cz == g.nz - 1) {
                for (int t = 0; t < 7; ++t)
                    if (!fits(g, cx, cy, cz, t + 1)) G[(int64_t)(1 + t) * V + xo] = CODE_NONE;
                for (int t = 0; t < 12; ++t)
                    if (!fits(g, cx, cy, cz, tri_step(t, 0) | tri_step(t, 1))) G[(int64_t)(8 + t) * V + xo] = CODE_NONE;
                for (int t = 0; t < 6; ++t) G[tet_code_at(V, xo, t)] = CODE_NONE;
            }
            if (lower) {
                star_cells(lower, own_lo, own_hi);
                ncell = (uint32_t)(popc64(own_lo) + __builtin_popcount(own_hi));
                uint64_t rp;
                relabel<PACKED>(r, lower, inv0, inv1, rp);
                // x pairs with its lowest edge (the code is known before the loop)
                G[xo] = (uint8_t)(13 + T.l27[inv0 & 15u]);
            } else {
                G[xo] = CODE_CRIT;  // minimum
            }
            stash[0 * GB + tid] = inv0;
            stash[1 * GB + tid] = inv1;
            stash[2 * GB + tid] = rv;
            stash[3 * GB + tid] = lower | own_hi << 16;
            stash[4 * GB + tid] = (uint32_t)own_lo;
            stash[5 * GB + tid] = (uint32_t)(own_lo >> 32);
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

    uint32_t inv0 = 0, inv1 = 0, lower = 0;
    uint64_t in_lo = 0;
    uint32_t in_hi = 0;
    if (active) {
        const int v = perm[tid];
        inv0 = stash[0 * GB + v];
        inv1 = stash[1 * GB + v];
        rx = stash[2 * GB + v];
        const uint32_t w3 = stash[3 * GB + v];
        lower = w3 & 0xFFFFu;
        in_hi = w3 >> 16;
        in_lo = stash[4 * GB + v] | (uint64_t)stash[5 * GB + v] << 32;
    }
    __syncthreads();  // the code buffer is written from here on
    if (active) {
        if (lower == 0) {
            crit_vertex = true;
        } else {
            const int k = __builtin_popcount(lower);
            // the largest k among the lanes here (k <= 14): the minimum
            // searches of the wave run that many levels in every lane, as
            // scalar branches
            int kw = 0;
#pragma unroll
            for (int step = 8; step >= 1; step >>= 1)
                if (__builtin_amdgcn_ballot_w64(k >= kw + step)) kw += step;
            kw = __builtin_amdgcn_readfirstlane(kw);
            uint8_t xcode;
            lower_star_gradient(
                T, in_lo, in_hi, kw, inv0, inv1, [&](int s, uint8_t code) { CODE(s) = code; }, xcode, crit_lo,
                crit_hi);
            // the labels again, for the keys of the critical cells (not kept
            // in registers through the loop)
            relpack = labels_of(inv0, inv1, k);
        }
    }
    __syncthreads();

    // ---- 3. gradient codes of the own vertex's lower star: one store per slot,
    // consecutive lanes -> consecutive bytes ----
    // The plane and the anchor offset of a slot are the same in every lane:
    // the address is a base common to the workgroup plus the lane's own
    // offset (tid bytes; 6 tid in the tetrahedron plane, 6 bytes per anchor).
    {
        const uint32_t col = own_lane;
        const uint32_t ve = tid, vt = 6 * tid;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            const bool w = s < 64 ? ((own_lo >> s) & 1) : ((own_hi >> (s - 64)) & 1);
            if (w) {
                constexpr int64_t zero = 0;
                const int pl = kStar.plane[s];  // compile-time after unrolling
                const int64_t a0 = x0 + (zero + kStar.aoff[s][0]) + kStar.aoff[s][1] * g.sy + kStar.aoff[s][2] * g.sz;
                uint8_t* const base = G + (pl < 20 ? (int64_t)pl * V + a0 : tet_code_at(V, a0, pl - 20));
                base[pl < 20 ? ve : vt] = scode[s * GB + col];
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
    if (g.V <= ((int64_t)1 << 28))  // ranks fit 28 bits: (rank << 4 | neighbour) sorts in 32 bits
        hipLaunchKernelGGL(k_gradient<true>, dim3((unsigned)blocks), dim3(GB), 0, st, g, rank, G, bpr, cl);
    else
        hipLaunchKernelGGL(k_gradient<false>, dim3((unsigned)blocks), dim3(GB), 0, st, g, rank, G, bpr, cl);
}

}  // namespace dms
