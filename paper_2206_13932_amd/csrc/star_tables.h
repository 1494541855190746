// Compile-time tables of the open star of a vertex in the Freudenthal/Kuhn
// triangulation (14 edges, 36 triangles, 24 tetrahedra around an interior
// vertex). Computed by constexpr code so that fully unrolled device loops
// fold them into immediates; the same values are also copied to LDS for
// lookups with per-lane indices.
#pragma once
#include "dms_device.h"

namespace dms {

struct StarBuild {
    StarTables t{};
    int ncell = 0;
    uint16_t le_nb[36]{};
    uint16_t lt_nb[24]{};
};

constexpr int nb_mask(int n) { return n < 7 ? n + 1 : n - 6; }
constexpr int nb_sign(int n) { return n < 7 ? 1 : -1; }
constexpr int nb_comp(int n, int a) { return nb_sign(n) * ((nb_mask(n) >> a) & 1); }
constexpr int nb_csum(int n) { return nb_comp(n, 0) + nb_comp(n, 1) + nb_comp(n, 2); }

constexpr bool nb_adjacent(int a, int b) {
    int d[3] = {nb_comp(a, 0) - nb_comp(b, 0), nb_comp(a, 1) - nb_comp(b, 1), nb_comp(a, 2) - nb_comp(b, 2)};
    bool pos = true, neg = true, nz = false;
    for (int i = 0; i < 3; ++i) {
        if (!(d[i] == 0 || d[i] == 1)) pos = false;
        if (!(d[i] == 0 || d[i] == -1)) neg = false;
        if (d[i] != 0) nz = true;
    }
    return nz && (pos || neg);
}

constexpr int ct_tri_type(int a, int b) {
    constexpr uint8_t t[12] = {0x21, 0x41, 0x61, 0x12, 0x42, 0x52, 0x43, 0x14, 0x24, 0x34, 0x25, 0x16};
    for (int i = 0; i < 12; ++i)
        if ((t[i] & 15) == a && (t[i] >> 4) == b) return i;
    return -1;
}
constexpr int ct_tet_type(int a, int b, int c) {
    constexpr uint16_t t[6] = {0x421, 0x241, 0x412, 0x142, 0x214, 0x124};
    for (int i = 0; i < 6; ++i)
        if ((t[i] & 15) == a && ((t[i] >> 4) & 15) == b && ((t[i] >> 8) & 15) == c) return i;
    return -1;
}

// Fill geometry of one slot from its neighbour set.
constexpr void fill_slot(StarTables& T, int s, uint16_t nbset) {
    // points of the simplex: x (origin) + neighbours; sort by coordinate sum
    int pts[4][3] = {};
    int np = 1;
    for (int n = 0; n < NNB; ++n)
        if (nbset & (1 << n)) {
            pts[np][0] = nb_comp(n, 0);
            pts[np][1] = nb_comp(n, 1);
            pts[np][2] = nb_comp(n, 2);
            ++np;
        }
    for (int i = 0; i < np; ++i)
        for (int j = i + 1; j < np; ++j) {
            int si = pts[i][0] + pts[i][1] + pts[i][2];
            int sj = pts[j][0] + pts[j][1] + pts[j][2];
            if (sj < si)
                for (int a = 0; a < 3; ++a) {
                    int tmp = pts[i][a];
                    pts[i][a] = pts[j][a];
                    pts[j][a] = tmp;
                }
        }
    int steps[3] = {};
    for (int i = 0; i + 1 < np; ++i) {
        int m = 0;
        for (int a = 0; a < 3; ++a)
            if (pts[i + 1][a] - pts[i][a] == 1) m |= 1 << a;
        steps[i] = m;
    }
    int dim = np - 1;
    int type = dim == 1 ? steps[0] - 1 : dim == 2 ? ct_tri_type(steps[0], steps[1]) : ct_tet_type(steps[0], steps[1], steps[2]);
    T.cellnb[s] = nbset;
    T.dim[s] = (uint8_t)dim;
    T.type[s] = (uint8_t)type;
    T.plane[s] = (uint8_t)(plane_base(dim) + type);
    for (int a = 0; a < 3; ++a) T.aoff[s][a] = (int8_t)pts[0][a];
    T.al27[s] = (int8_t)(pts[0][0] + 3 * pts[0][1] + 9 * pts[0][2]);
}

constexpr StarTables make_star_tables() {
    StarTables T{};
    for (int n = 0; n < NNB; ++n) {
        for (int a = 0; a < 3; ++a) T.nbv[n][a] = (int8_t)nb_comp(n, a);
        T.l27[n] = (int8_t)(nb_comp(n, 0) + 3 * nb_comp(n, 1) + 9 * nb_comp(n, 2));
        uint16_t lc = 0;
        for (int m = 0; m < NNB; ++m)
            if (nb_csum(m) < nb_csum(n)) lc |= (uint16_t)(1 << m);
        T.lessc[n] = lc;
        T.cpos_pos[n] = nb_csum(n) > 0 ? 1 : 0;
    }
    int s = 0;
    for (int n = 0; n < NNB; ++n) fill_slot(T, s++, (uint16_t)(1 << n));
    for (int a = 0; a < NNB; ++a)
        for (int b = a + 1; b < NNB; ++b)
            if (nb_adjacent(a, b)) fill_slot(T, s++, (uint16_t)((1 << a) | (1 << b)));
    for (int a = 0; a < NNB; ++a)
        for (int b = a + 1; b < NNB; ++b)
            for (int c = b + 1; c < NNB; ++c)
                if (nb_adjacent(a, b) && nb_adjacent(a, c) && nb_adjacent(b, c))
                    fill_slot(T, s++, (uint16_t)((1 << a) | (1 << b) | (1 << c)));
    for (int i = 0; i < NSLOT; ++i) {
        T.face[i] = 0;
        T.cofc[i] = 0;
    }
    for (int i = 0; i < NSLOT; ++i) T.slrec[i] = (uint32_t)T.cellnb[i] | (uint32_t)(T.al27[i] + 13) << 16;
    for (int n = 0; n < NNB; ++n)
        T.nbrec[n] = (uint32_t)T.lessc[n] | (uint32_t)T.cpos_pos[n] << 14 | (uint32_t)(T.l27[n] + 13) << 16;
    for (int n = 0; n < 16; ++n) {  // cellnb has 14 bits: rows 14 and 15 stay empty
        T.slnb[n] = SlotMask{0, 0, 0};
        T.slnbc[2 * n] = 0;
        T.slnbc[2 * n + 1] = 0;
        for (int i = 0; i < NSLOT; ++i)
            if (T.cellnb[i] & (1 << n)) {
                if (i < 64) T.slnb[n].lo |= (uint64_t)1 << i;
                else T.slnb[n].hi |= 1u << (i - 64);
                if (i >= NNB) T.slnbc[2 * n] |= (uint64_t)1 << (i - NNB);
            }
    }
    for (int i = 0; i < NSLOT; ++i)
        for (int j = 0; j < NSLOT; ++j) {
            if (T.dim[j] != T.dim[i] + 1) continue;
            if ((T.cellnb[i] & T.cellnb[j]) != T.cellnb[i]) continue;
            // j is a cofacet of i, i a facet of j
            T.face[j] |= (uint64_t)1 << i;   // facets always sit below slot 64
            T.cofc[i] |= (uint64_t)1 << (j - NNB);  // cofacets always sit at slot 14 or above
        }
    return T;
}

constexpr StarTables kStar = make_star_tables();

static_assert(kStar.dim[13] == 1 && kStar.dim[14] == 2 && kStar.dim[49] == 2 && kStar.dim[50] == 3 &&
                  kStar.dim[73] == 3,
              "slot layout: 14 edges, 36 triangles, 24 tetrahedra");

}  // namespace dms
