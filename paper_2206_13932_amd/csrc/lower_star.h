// ProcessLowerStars on one vertex (Robins et al., as the paper's Alg.
// "Zero-persistence skip" and Sec. 2.6 use it), written for one GPU lane.
//
// Notation. x is the vertex, its lower neighbours are relabelled 0..k-1 by
// rank (the label of a neighbour is its place among them), and a cell of the
// lower star L(x) is the set of its lower neighbours. The lexicographic order
// of Sec. 2.2 restricted to L(x) is the integer order of the cells' label
// bitmasks: the highest differing vertex decides, and a face is a mask that
// lacks only lower bits.
//
// Cells are the 74 slots of the open star (star_tables.h); both priority
// queues are slot sets. The minimum of a set is found by elimination from
// the highest label down: at label j, if some member lacks j, the members
// that hold j go; the last member standing has the smallest mask. The slots
// holding a neighbour are one table row, so a level costs a few bit
// operations whatever the set's size.
#pragma once
#include "dms_device.h"

namespace dms {

// ---- Batcher's odd-even merge sort on 16 keys (63 compare-exchanges) ----
struct SortNet16 {
    uint8_t a[64], b[64];
    int n = 0;
};
constexpr SortNet16 make_sortnet16() {
    SortNet16 s{};
    // iterative form of Batcher's network for N = 16
    for (int p = 1; p < 16; p <<= 1)
        for (int k = p; k >= 1; k >>= 1)
            for (int j = k % p; j + k < 16; j += 2 * k)
                for (int i = 0; i < k && i + j + k < 16; ++i)
                    if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        s.a[s.n] = (uint8_t)(i + j);
                        s.b[s.n] = (uint8_t)(i + j + k);
                        ++s.n;
                    }
    return s;
}
constexpr SortNet16 kSortNet16 = make_sortnet16();
static_assert(kSortNet16.n == 63, "Batcher's network on 16 keys has 63 comparators");

// Labels of the lower neighbours from their ranks r[n] (lower: bit n set).
// Out: inv0 / inv1 = the neighbour holding label j, 4 bits per label (labels
// 0..7, then 8..13; 15 for a label past the last lower neighbour); relpack =
// the label of neighbour n at bits 4n (lower neighbours only). PACKED: ranks
// below 2^28, so (rank << 4 | n) sorts in 32 bits; otherwise each label is
// counted.
template <bool PACKED>
__host__ __device__ inline void relabel(const uint32_t (&r)[NNB], uint32_t lower, uint32_t& inv0, uint32_t& inv1,
                                        uint64_t& relpack) {
    inv0 = 0;
    inv1 = 0;
    relpack = 0;
    if (PACKED) {
        uint32_t a[16];
#pragma unroll
        for (int n = 0; n < NNB; ++n) a[n] = ((lower >> n) & 1) ? (r[n] << 4) | (uint32_t)n : 0xFFFFFFFFu;
        a[14] = 0xFFFFFFFFu;
        a[15] = 0xFFFFFFFFu;
#pragma unroll
        for (int c = 0; c < kSortNet16.n; ++c) {
            const uint32_t u = a[kSortNet16.a[c]], v = a[kSortNet16.b[c]];
            a[kSortNet16.a[c]] = u < v ? u : v;
            a[kSortNet16.b[c]] = u < v ? v : u;
        }
#pragma unroll
        for (int j = 0; j < NNB; ++j) {
            const uint32_t n = a[j] & 15u;  // 15 past the last lower neighbour
            if (j < 8) inv0 |= n << (4 * j);
            else inv1 |= n << (4 * (j - 8));
            if (a[j] != 0xFFFFFFFFu) relpack |= (uint64_t)j << (4 * n);
        }
    } else {
#pragma unroll
        for (int n = 0; n < NNB; ++n) {
            uint32_t c = 0;
#pragma unroll
            for (int m = 0; m < NNB; ++m)
                if (m != n) c += ((lower >> m) & 1) && r[m] < r[n];
            if ((lower >> n) & 1) {
                relpack |= (uint64_t)c << (4 * n);
                if (c < 8) inv0 |= (uint32_t)n << (4 * c);
                else inv1 |= (uint32_t)n << (4 * (c - 8));
            }
        }
        const uint64_t past = ((1ull << (4 * NNB)) - 1) & ~((1ull << (4 * __builtin_popcount(lower))) - 1);
        inv0 |= (uint32_t)past;
        inv1 |= (uint32_t)(past >> 32);
    }
}

// The cells of L(x): every slot minus those holding a neighbour that is not
// lower (or not in the grid).
__host__ __device__ inline void star_cells(uint32_t lower, uint64_t& in_lo, uint32_t& in_hi) {
    uint64_t rm_lo = 0;
    uint32_t rm_hi = 0;
#pragma unroll
    for (int n = 0; n < NNB; ++n)
        if (!((lower >> n) & 1)) {
            rm_lo |= kStar.slnb[n].lo;
            rm_hi |= kStar.slnb[n].hi;
        }
    in_lo = ~rm_lo;
    in_hi = ((1u << (NSLOT - 64)) - 1) & ~rm_hi;
}

__host__ __device__ inline int popc64_(uint64_t v) { return __builtin_popcountll(v); }

// The label of each lower neighbour (bits 4n) from inv0 / inv1.
__host__ __device__ inline uint64_t labels_of(uint32_t inv0, uint32_t inv1, int k) {
    const uint64_t inv = inv0 | (uint64_t)inv1 << 32;
    uint64_t relpack = 0;
#pragma unroll
    for (int j = 0; j < NNB; ++j)
        if (j < k) relpack |= (uint64_t)j << (4 * ((inv >> (4 * j)) & 15u));
    return relpack;
}

// ProcessLowerStars on a vertex with k >= 1 lower neighbours.
// T: star tables (face, cofc, slrec, nbrec, l27, cpos_pos, slnb, slnbc);
// inv0 / inv1 as relabel leaves them (15 past label k-1); levels: the number
// of labels the minimum searches go through, at least k (lanes that run in
// lock-step pass the largest k among them, so that the searches' levels are
// the same in every lane: a level past a lane's own labels reads the empty
// row 15 of slnb and changes nothing);
// put(slot, code) receives the partner code of every cell
// of L(x) that is paired (codes as in dms_device.h); xcode = the code of x;
// crit_lo / crit_hi = the critical cells.
template <class Tab, class Put>
__host__ __device__ inline void lower_star_gradient(const Tab& T, uint64_t in_lo, uint32_t in_hi, int levels,
                                                    uint32_t inv0, uint32_t inv1, Put put, uint8_t& xcode,
                                                    uint64_t& crit_lo, uint32_t& crit_hi) {
    auto nb_of = [&](int j) __attribute__((always_inline)) { return (int)((j < 8 ? inv0 >> (4 * j) : inv1 >> (4 * (j - 8))) & 15u); };
    crit_lo = 0;
    crit_hi = 0;
    // classified cells; the slots outside L(x) count as classified from the
    // start, so that no test needs the star's mask again
    uint64_t cls_lo;
    uint32_t cls_hi = ~in_hi;
    // pair (p, a): p is a facet of a; w = the neighbour of a not in p
    auto pair_cells = [&](int p, int a) __attribute__((always_inline)) {
        const uint32_t ra = T.slrec[a], rp = T.slrec[p];
        const uint32_t w = __builtin_ctz(ra & ~rp & 0x3FFFu);
        const uint32_t rw = T.nbrec[w];
        const int pos = __builtin_popcount(ra & rw & 0x3FFFu) + (int)((rw >> 14) & 1);
        put(a, (uint8_t)(0x80 | pos));
        put(p, (uint8_t)(13 + (int)(rw >> 16) - (int)(rp >> 16)));  // 13 + l27[w] - al27[p]
    };
    // x pairs with its lowest edge delta = {x, n0}
    const int n0 = nb_of(0);
    xcode = (uint8_t)(13 + T.l27[n0]);
    put(n0, (uint8_t)(0x80 | T.cpos_pos[n0]));
    cls_lo = ~in_lo | (uint64_t)1 << n0;
    uint64_t z_lo = 0x3FFFull & ~cls_lo;  // the other edges
    uint32_t z_hi = 0;
    // Cofacets are triangles and tetrahedra (slots 14..73): sets of them are
    // one word, bit s - 14 ("cofacet words"). The first queue only ever holds
    // cofacets.
    uint64_t o = 0;
    auto cof_word = [](uint64_t lo, uint32_t hi) __attribute__((always_inline)) {
        return lo >> NNB | (uint64_t)hi << (64 - NNB);
    };
    // the classified cells among them (those outside L(x) count as classified)
    uint64_t cls_c = ~cof_word(in_lo, in_hi);
    // The unpaired (unclassified) facets of every cofacet slot, a 2-bit count
    // kept in two bit planes of cofacet words (u0: bit 0, u1: bit 1). The
    // facets inside the star of a cell of L(x) are cells of L(x): 2 for a
    // triangle, 3 for a tetrahedron (x itself is paired apart). The counts of
    // slots outside L(x) are never read (those slots count as classified).
    uint64_t u0 = ~((1ull << (50 - NNB)) - 1), u1 = ~0ull;
    // m: the cofacets of the cells just classified (the cofacets of a cell
    // and of its facet are disjoint, so every count drops by one). Those
    // still unclassified go to the queue their count now names: one unpaired
    // facet -> o, none -> z (and out of o). A cell with none left was pushed
    // to o when it had one; it would leave o for z when popped, with no other
    // effect, so it moves there now and costs no pop.
    auto push_cofaces = [&](uint64_t m) __attribute__((always_inline)) {
        u1 ^= m & ~u0;
        u0 ^= m;
        const uint64_t c = m & ~cls_c & ~u1;  // count 0 or 1
        const uint64_t none = c & ~u0;
        o = (o | c) & ~none;
        z_lo |= none << NNB;
        z_hi |= (uint32_t)(none >> (64 - NNB));
    };
    // The member of a non-empty set with the smallest mask is what is left
    // after the levels: a set of one bit. Every level runs: the lanes of a
    // wave go through the levels together, and testing after each level
    // whether one member is left cost more than the levels it saved. The rows
    // of label j sit at byte offset 16 n(j) of slnb and of slnbc; the offsets
    // are kept one byte per label, so that a level takes its row's address
    // with one bit-field extract.
    static_assert(sizeof(SlotMask) == 16, "one slnb row is 16 bytes");
    uint32_t roff[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t q = (w < 2 ? inv0 >> (16 * w) : inv1 >> (16 * (w - 2))) & 0xFFFFu;
        roff[w] = (q & 0xFu) << 4 | (q & 0xF0u) << 8 | (q & 0xF00u) << 12 | (q & 0xF000u) << 16;
    }
    auto row_off = [&](int j) __attribute__((always_inline)) { return (roff[j >> 2] >> (8 * (j & 3))) & 0xFFu; };
    const char* const rows = (const char*)&T.slnb[0];
    const char* const rows_c = (const char*)&T.slnbc[0];
    auto min_of = [&](uint64_t& lo, uint32_t& hi) __attribute__((always_inline)) {
        if (popc64_(lo) + __builtin_popcount(hi) > 1) {
#pragma unroll
            for (int j = NNB - 1; j >= 0; --j) {
                if (j < levels) {
                    const SlotMask m = *(const SlotMask*)(rows + row_off(j));
                    const uint64_t tl = lo & ~m.lo;
                    const uint32_t th = hi & ~m.hi;
                    if (tl | th) {
                        lo = tl;
                        hi = th;
                    }
                }
            }
        }
    };
    auto min_of_cof = [&](uint64_t q) __attribute__((always_inline)) {
        if (popc64_(q) > 1) {
#pragma unroll
            for (int j = NNB - 1; j >= 0; --j) {
                if (j < levels) {
                    const uint64_t t = q & ~*(const uint64_t*)(rows_c + row_off(j));
                    if (t) q = t;
                }
            }
        }
        return q;
    };
    push_cofaces(T.cofc[n0]);
    for (int guard = 0; guard < 4 * NSLOT; ++guard) {
        while (o) {
            const uint64_t ab = min_of_cof(o);
            o ^= ab;
            const int a = NNB + __builtin_ctzll(ab);
            // A cell of this queue is unclassified (it is smaller than every
            // cell classified after it entered), and it has one unpaired facet
            // (the classification that takes its last one moves it to the other
            // queue), so it pairs with that facet.
            const int p = __builtin_ctzll(T.face[a] & ~cls_lo);
            pair_cells(p, a);
            cls_lo |= ab << NNB | (uint64_t)1 << p;
            cls_hi |= (uint32_t)(ab >> (64 - NNB));
            cls_c |= ab | (p >= NNB ? (uint64_t)1 << (p - NNB) : 0);
            z_lo &= ~((uint64_t)1 << p);
            push_cofaces(T.cofc[a] | T.cofc[p]);
        }
        if (!(z_lo | z_hi)) break;
        uint64_t clo = z_lo;
        uint32_t chi = z_hi;
        min_of(clo, chi);
        const int c = clo ? __builtin_ctzll(clo) : 64 + __builtin_ctz(chi);
        z_lo ^= clo;
        z_hi ^= chi;
        cls_lo |= clo;
        cls_hi |= chi;
        cls_c |= cof_word(clo, chi);
        crit_lo |= clo;
        crit_hi |= chi;
        put(c, CODE_CRIT);
        push_cofaces(T.cofc[c]);
    }
}

}  // namespace dms
