// Host build of the GPU gradient kernel's per-vertex routine, for CPU tests.
//
// The routine (relabel, star_cells, lower_star_gradient in lower_star.h, on the
// star tables of star_tables.h) is compiled for the host and run on every
// vertex of a small grid, one vertex after another, with the same inputs the
// kernel gives it: the 14-bit mask of lower neighbours (a neighbour outside
// the grid is not lower), the labels from the rank sort, and a number of
// minimum-search levels of at least the vertex's own lower-star size.
// Every cell code goes to the gradient byte planes (26 planes of V bytes; the
// tetrahedra as planes too, the layout the library's debug copy hands out),
// so the tests decode them exactly like the GPU's.
//
// This file is test infrastructure: it shares nothing with the oracle, which
// the tests compare it against.
#include <cstdint>
#include <cstring>

#include "star_tables.h"
#include "lower_star.h"

using namespace dms;

namespace {

constexpr uint8_t NEVER = 0xEE;  // a byte no cell of a lower star may keep

// levels_mode: 0 = the vertex's own lower-star size k, 1 = all 14 labels,
// 2 = k plus a pseudo-random number of extra levels (lanes of one wave pass
// the largest k among them)
template <bool PACKED>
int run(int nx, int ny, int nz, const uint32_t* rank, uint32_t offset, int levels_mode, uint8_t* G,
        int64_t* crit) {
    const int64_t V = (int64_t)nx * ny * nz;
    std::memset(G, NEVER, (size_t)PLANES * V);
    for (int d = 0; d < 4; ++d) crit[d] = 0;
    uint32_t lcg = 12345u;
    for (int64_t x = 0; x < V; ++x) {
        const int cx = (int)(x % nx), cy = (int)((x / nx) % ny), cz = (int)(x / ((int64_t)nx * ny));
        const uint32_t rv = rank[x] + offset;
        uint32_t r[NNB];
        uint32_t lower = 0;
        for (int n = 0; n < NNB; ++n) {
            const int ax = cx + kStar.nbv[n][0], ay = cy + kStar.nbv[n][1], az = cz + kStar.nbv[n][2];
            const bool in = ax >= 0 && ax < nx && ay >= 0 && ay < ny && az >= 0 && az < nz;
            r[n] = in ? rank[ax + (int64_t)nx * (ay + (int64_t)ny * az)] + offset : 0xFFFFFFFFu;
            if (in && r[n] < rv) lower |= 1u << n;
        }
        if (!lower) {  // a minimum: x is critical, its star holds no other cell
            G[x] = CODE_CRIT;
            ++crit[0];
            continue;
        }
        uint64_t in_lo;
        uint32_t in_hi;
        star_cells(lower, in_lo, in_hi);
        uint32_t inv0, inv1;
        uint64_t relpack;
        relabel<PACKED>(r, lower, inv0, inv1, relpack);
        const int k = __builtin_popcount(lower);
        if (labels_of(inv0, inv1, k) != relpack) return 1;  // the two label forms disagree
        G[x] = (uint8_t)(13 + kStar.l27[inv0 & 15u]);
        int levels = k;
        if (levels_mode == 1) levels = NNB;
        if (levels_mode == 2) {
            lcg = lcg * 1664525u + 1013904223u;
            levels = k + (int)((lcg >> 24) % (uint32_t)(NNB - k + 1));
        }
        uint8_t code[NSLOT];
        std::memset(code, NEVER, sizeof code);
        uint8_t xcode = 0;
        uint64_t clo = 0;
        uint32_t chi = 0;
        lower_star_gradient(
            kStar, in_lo, in_hi, levels, inv0, inv1, [&](int s, uint8_t c) { code[s] = c; }, xcode, clo, chi);
        if (xcode != G[x]) return 2;  // the routine's code of x differs from the kernel's
        for (int s = 0; s < NSLOT; ++s) {
            const bool in = s < 64 ? ((in_lo >> s) & 1) : ((in_hi >> (s - 64)) & 1);
            if (!in) {
                if (code[s] != NEVER) return 3;  // a code for a cell outside the lower star
                continue;
            }
            if (code[s] == NEVER) return 4;  // a cell of the lower star without a code
            const int64_t a = x + kStar.aoff[s][0] + (int64_t)nx * (kStar.aoff[s][1] + (int64_t)ny * kStar.aoff[s][2]);
            G[(int64_t)kStar.plane[s] * V + a] = code[s];
            const bool c = s < 64 ? ((clo >> s) & 1) : ((chi >> (s - 64)) & 1);
            if (c != (code[s] == CODE_CRIT)) return 5;  // critical list and codes disagree
            if (c) ++crit[kStar.dim[s]];
        }
    }
    return 0;
}

}  // namespace

extern "C" int ls_host_gradient(int nx, int ny, int nz, const uint32_t* rank, uint32_t offset, int packed,
                                int levels_mode, uint8_t* G, int64_t* crit) {
    if (nx < 2 || ny < 2 || nz < 2) return -1;
    const int64_t V = (int64_t)nx * ny * nz;
    if ((uint64_t)offset + (uint64_t)V >= (packed ? (1ull << 28) : 0xFFFFFFFFull)) return -1;
    return packed ? run<true>(nx, ny, nz, rank, offset, levels_mode, G, crit)
                  : run<false>(nx, ny, nz, rank, offset, levels_mode, G, crit);
}

// The rank sort's network (kSortNet16) against the 0-1 principle: a
// comparator network sorts every input if it sorts every input of zeros and
// ones, so all 2^16 of them are run. Returns the number that come out
// unsorted.
extern "C" int ls_host_sortnet_01() {
    int bad = 0;
    for (uint32_t bits = 0; bits < (1u << 16); ++bits) {
        uint32_t a[16];
        for (int i = 0; i < 16; ++i) a[i] = (bits >> i) & 1u;
        for (int c = 0; c < kSortNet16.n; ++c) {
            const uint32_t u = a[kSortNet16.a[c]], v = a[kSortNet16.b[c]];
            a[kSortNet16.a[c]] = u < v ? u : v;
            a[kSortNet16.b[c]] = u < v ? v : u;
        }
        for (int i = 0; i + 1 < 16; ++i)
            if (a[i] > a[i + 1]) {
                ++bad;
                break;
            }
    }
    return bad;
}
