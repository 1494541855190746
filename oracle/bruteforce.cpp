/*
 * BRUTE-FORCE CHECKER -- TEST INFRASTRUCTURE ONLY.
 *
 * Pins the oracle against the plain definition of persistence. It shares no
 * code with the oracle: simplices are enumerated from the tetrahedra down
 * (every face of every Kuhn tetrahedron), not from the oracle's id tables.
 *
 *  - bf_diagram: the whole lexicographic filtration (Sec. 2.2), reduced by
 *    Z2 column reduction (PairSimplices is boundary-matrix reduction,
 *    Sec. 2.5), with clearing (dimension separability, Sec. 4.1(a)). Pairs
 *    are reported in vertex-order space: (dim, rank of the birth simplex's
 *    highest vertex, rank of the death simplex's highest vertex); pairs of
 *    zero persistence (same highest vertex) are dropped, since the method
 *    skips exactly those (Sec. 4.1(c)).
 *  - bf_lower_link_betti: reduced Betti numbers of the lower link of every
 *    vertex; the expansion-based gradient has exactly that many critical
 *    cells per dimension in each lower star (Sec. 1.1, Sec. 2.6).
 *  - bf_counts: numbers of vertices, edges, triangles and tetrahedra.
 *  - bf_d0_kruskal / bf_d2_dual: D0 and D2 of the whole filtration from
 *    union-finds over every edge, or over every triangle and tetrahedron
 *    with the outside (Sec. 5.1, 5.2), cheap enough for 512^3 grids.
 *  - bf_check_cycles: persistent 1-cycle generators against their
 *    definition (Sec. 8).
 * A grid with nz = 1 is the 2D grid of the plane z = 0, built from its
 * triangles (there the lower link of a vertex is a graph).
 */
#include <algorithm>
#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <vector>

namespace {

typedef int64_t i64;
typedef std::array<i64, 4> Verts;  /* ascending vertex ids, padded with -1 at the end */

struct Complex {
    std::vector<Verts> simp;
    std::vector<int> dim;
};

/* Kuhn triangulation: each unit cube is cut into the 6 monotone lattice
 * paths from its lowest to its highest corner. */
void tetrahedra(i64 nx, i64 ny, i64 nz, std::vector<std::array<i64, 4>>& tets) {
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    tets.clear();
    for (i64 z = 0; z + 1 < nz; ++z)
        for (i64 y = 0; y + 1 < ny; ++y)
            for (i64 x = 0; x + 1 < nx; ++x)
                for (int p = 0; p < 6; ++p) {
                    i64 c[3] = {x, y, z};
                    std::array<i64, 4> t;
                    t[0] = c[0] + nx * (c[1] + ny * c[2]);
                    for (int s = 0; s < 3; ++s) {
                        c[perm[p][s]] += 1;
                        t[s + 1] = c[0] + nx * (c[1] + ny * c[2]);
                    }
                    std::sort(t.begin(), t.end());
                    tets.push_back(t);
                }
}

/* A 2D grid (nz = 1): each unit square is cut into the 2 monotone lattice
 * paths from its lowest to its highest corner (the same triangulation the
 * plane z = 0 receives from the 3D one). Padded with -1. */
void triangles2d(i64 nx, i64 ny, std::vector<std::array<i64, 4>>& tris) {
    tris.clear();
    for (i64 y = 0; y + 1 < ny; ++y)
        for (i64 x = 0; x + 1 < nx; ++x) {
            const i64 a = x + nx * y, b = a + 1, c = a + nx, d = a + nx + 1;
            tris.push_back({a, b, d, -1});
            tris.push_back({a, c, d, -1});
        }
}

void all_simplices(i64 nx, i64 ny, i64 nz, Complex& K) {
    std::vector<std::array<i64, 4>> tops;
    if (nz == 1) triangles2d(nx, ny, tops);
    else tetrahedra(nx, ny, nz, tops);
    const int nv = nz == 1 ? 3 : 4;
    std::set<Verts> seen;
    for (auto& t : tops)
        for (int m = 1; m < (1 << nv); ++m) {
            Verts v = {-1, -1, -1, -1};
            int k = 0;
            for (int i = 0; i < nv; ++i)
                if (m & (1 << i)) v[k++] = t[i];
            std::sort(v.begin(), v.begin() + k);
            seen.insert(v);
        }
    K.simp.assign(seen.begin(), seen.end());
    K.dim.resize(K.simp.size());
    for (size_t i = 0; i < K.simp.size(); ++i) {
        int d = -1;
        for (int j = 0; j < 4; ++j) d += (K.simp[i][j] >= 0);
        K.dim[i] = d;
    }
}

/* sorted-decreasing ranks padded with -1: the lexicographic comparison */
std::array<i64, 4> lex_key(const Verts& v, const uint32_t* rank) {
    std::array<i64, 4> k = {-1, -1, -1, -1};
    int n = 0;
    for (int i = 0; i < 4; ++i)
        if (v[i] >= 0) k[n++] = rank[v[i]];
    std::sort(k.begin(), k.begin() + n, [](i64 a, i64 b) { return a > b; });
    return k;
}

void sym_diff(std::vector<int>& a, const std::vector<int>& b, std::vector<int>& tmp) {
    tmp.clear();
    size_t i = 0, j = 0;
    while (i < a.size() || j < b.size()) {
        if (j == b.size() || (i < a.size() && a[i] < b[j])) tmp.push_back(a[i++]);
        else if (i == a.size() || b[j] < a[i]) tmp.push_back(b[j++]);
        else { ++i; ++j; }
    }
    a.swap(tmp);
}

}  // namespace

extern "C" {

int64_t bf_counts(int64_t nx, int64_t ny, int64_t nz, int64_t* counts4) {
    Complex K;
    all_simplices(nx, ny, nz, K);
    for (int d = 0; d < 4; ++d) counts4[d] = 0;
    for (int d : K.dim) counts4[d]++;
    return (int64_t)K.simp.size();
}

/* Output: finite pairs as (dim, birth rank, death rank) triples into pairs
 * (capacity cap triples), essential classes as (dim, birth rank) into ess
 * (capacity cap_e). Returns the number of finite pairs with positive
 * persistence; *n_ess receives the number of essential classes. */
int64_t bf_diagram(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t* pairs,
                   int64_t cap, int64_t* ess, int64_t cap_e, int64_t* n_ess) {
    Complex K;
    all_simplices(nx, ny, nz, K);
    const size_t n = K.simp.size();
    std::vector<std::array<i64, 4>> key(n);
    for (size_t i = 0; i < n; ++i) key[i] = lex_key(K.simp[i], rank);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int> pos(n);
    for (size_t i = 0; i < n; ++i) pos[order[i]] = (int)i;
    std::map<Verts, int> index;
    for (size_t i = 0; i < n; ++i) index[K.simp[i]] = (int)i;

    /* columns in filtration order, rows = filtration positions of facets */
    std::vector<std::vector<int>> col(n);
    for (size_t j = 0; j < n; ++j) {
        int s = order[j];
        int d = K.dim[s];
        if (d == 0) continue;
        for (int drop = 0; drop <= d; ++drop) {
            Verts f = {-1, -1, -1, -1};
            int k = 0;
            for (int i = 0; i <= d; ++i)
                if (i != drop) f[k++] = K.simp[s][i];
            col[j].push_back(pos[index.at(f)]);
        }
        std::sort(col[j].begin(), col[j].end());
    }
    std::vector<int> owner(n, -1);    /* row -> column whose reduced pivot it is */
    std::vector<char> cleared(n, 0);  /* column known to reduce to zero */
    std::vector<char> is_birth(n, 0), is_death(n, 0);
    std::vector<int> tmp;
    std::vector<std::array<i64, 3>> out;
    for (int d = 3; d >= 1; --d) {
        for (size_t j = 0; j < n; ++j) {
            if (K.dim[order[j]] != d) continue;
            if (cleared[j]) { col[j].clear(); continue; }
            std::vector<int>& c = col[j];
            while (!c.empty() && owner[c.back()] >= 0) sym_diff(c, col[owner[c.back()]], tmp);
            if (c.empty()) continue;
            int low = c.back();
            owner[low] = (int)j;
            cleared[low] = 1;
            is_birth[low] = 1;
            is_death[j] = 1;
            i64 b = key[order[low]][0], e = key[order[j]][0];
            if (b != e) out.push_back({d - 1, b, e});
        }
    }
    std::sort(out.begin(), out.end());
    int64_t m = (int64_t)out.size();
    for (int64_t i = 0; i < m && i < cap; ++i)
        for (int k = 0; k < 3; ++k) pairs[i * 3 + k] = out[i][k];
    std::vector<std::array<i64, 2>> es;
    for (size_t i = 0; i < n; ++i)
        if (!is_birth[i] && !is_death[i]) es.push_back({K.dim[order[i]], key[order[i]][0]});
    std::sort(es.begin(), es.end());
    *n_ess = (int64_t)es.size();
    for (size_t i = 0; i < es.size() && (int64_t)i < cap_e; ++i) {
        ess[i * 2] = es[i][0];
        ess[i * 2 + 1] = es[i][1];
    }
    return m;
}

/* Reduced Betti numbers (b~_{-1}, b~_0, b~_1, b~_2) of the lower link of
 * every vertex: the link of x is the set of faces, opposite to x, of the
 * tetrahedra around x; the lower link keeps those whose vertices are all
 * lower than x. */
/* 2D grid: the link of x is the cycle of edges opposite x in its
 * triangles; the lower link is a graph, so b~_1 = E - V + components. */
static void lower_link_betti_2d(int64_t nx, int64_t ny, const uint32_t* rank, int32_t* out) {
    std::vector<std::array<i64, 4>> tris;
    triangles2d(nx, ny, tris);
    const i64 V = nx * ny;
    std::vector<std::vector<int>> around(V);
    for (size_t t = 0; t < tris.size(); ++t)
        for (int i = 0; i < 3; ++i) around[tris[t][i]].push_back((int)t);
    for (i64 x = 0; x < V; ++x) {
        std::set<i64> lv;
        std::set<std::pair<i64, i64>> le;
        for (int t : around[x]) {
            i64 o[2];
            int k = 0;
            for (int i = 0; i < 3; ++i)
                if (tris[t][i] != x) o[k++] = tris[t][i];
            const bool l0 = rank[o[0]] < rank[x], l1 = rank[o[1]] < rank[x];
            if (l0) lv.insert(o[0]);
            if (l1) lv.insert(o[1]);
            if (l0 && l1) le.insert({std::min(o[0], o[1]), std::max(o[0], o[1])});
        }
        int32_t* b = out + 4 * x;
        b[3] = 0;
        b[0] = lv.empty() ? 1 : 0;
        if (lv.empty()) { b[1] = b[2] = 0; continue; }
        std::map<i64, i64> par;
        for (i64 v : lv) par[v] = v;
        auto find = [&](i64 v) {
            while (par[v] != v) v = par[v] = par[par[v]];
            return v;
        };
        i64 comps = (i64)lv.size();
        for (auto& e : le) {
            i64 a = find(e.first), bb = find(e.second);
            if (a != bb) { par[a] = bb; --comps; }
        }
        b[1] = (int32_t)(comps - 1);
        b[2] = (int32_t)((i64)le.size() - (i64)lv.size() + comps);
    }
}

void bf_lower_link_betti(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int32_t* out) {
    if (nz == 1) {
        lower_link_betti_2d(nx, ny, rank, out);
        return;
    }
    std::vector<std::array<i64, 4>> tets;
    tetrahedra(nx, ny, nz, tets);
    const i64 V = nx * ny * nz;
    std::vector<std::vector<int>> around(V);
    for (size_t t = 0; t < tets.size(); ++t)
        for (int i = 0; i < 4; ++i) around[tets[t][i]].push_back((int)t);
    for (i64 x = 0; x < V; ++x) {
        std::set<i64> lv;
        std::set<std::pair<i64, i64>> le;
        std::set<std::array<i64, 3>> lt;
        bool interior = true;
        i64 c[3] = {x % nx, (x / nx) % ny, x / (nx * ny)};
        i64 n[3] = {nx, ny, nz};
        for (int a = 0; a < 3; ++a) interior = interior && c[a] > 0 && c[a] + 1 < n[a];
        for (int t : around[x]) {
            std::array<i64, 3> o;
            int k = 0;
            for (int i = 0; i < 4; ++i)
                if (tets[t][i] != x) o[k++] = tets[t][i];
            bool l[3];
            for (int i = 0; i < 3; ++i) l[i] = rank[o[i]] < rank[x];
            for (int i = 0; i < 3; ++i)
                if (l[i]) lv.insert(o[i]);
            for (int i = 0; i < 3; ++i)
                for (int j = i + 1; j < 3; ++j)
                    if (l[i] && l[j]) le.insert({o[i], o[j]});
            if (l[0] && l[1] && l[2]) lt.insert(o);
        }
        int32_t* b = out + 4 * x;
        b[0] = lv.empty() ? 1 : 0;
        if (lv.empty()) { b[1] = b[2] = b[3] = 0; continue; }
        std::map<i64, i64> par;
        for (i64 v : lv) par[v] = v;
        auto find = [&](i64 v) {
            while (par[v] != v) v = par[v] = par[par[v]];
            return v;
        };
        i64 comps = (i64)lv.size();
        for (auto& e : le) {
            i64 a = find(e.first), bb = find(e.second);
            if (a != bb) { par[a] = bb; --comps; }
        }
        /* whole link of an interior vertex = a 2-sphere: b2 = 1, else 0 */
        i64 full = 0;
        for (int t : around[x]) { (void)t; ++full; }
        int b2 = (interior && (i64)lt.size() == full) ? 1 : 0;
        i64 chi = (i64)lv.size() - (i64)le.size() + (i64)lt.size();
        b[1] = (int32_t)(comps - 1);
        b[2] = (int32_t)(comps - chi + b2);
        b[3] = b2;
    }
}

}  // extern "C"

extern "C" {

/* D0 in vertex-order space from the plain definition: Kruskal over every
 * edge of the triangulation in lexicographic order, with the elder rule
 * (the younger of two merging components dies). PairSimplices restricted to
 * dimension 0 is exactly this union-find (Sec. 2.5). Edges are enumerated
 * from vertex pairs whose coordinates differ by a non-zero 0/1 vector, not
 * from any id table. Output: (birth rank, death rank) of every pair with
 * positive persistence, sorted; returns their number. */
int64_t bf_d0_kruskal(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t* out, int64_t cap) {
    const int64_t V = nx * ny * nz;
    std::vector<uint64_t> keys;
    keys.reserve((size_t)(7 * V));
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                const int64_t v = x + nx * (y + ny * z);
                for (int m = 1; m < 8; ++m) {
                    const int64_t dx = m & 1, dy = (m >> 1) & 1, dz = (m >> 2) & 1;
                    if (x + dx >= nx || y + dy >= ny || z + dz >= nz) continue;
                    const int64_t w = (x + dx) + nx * ((y + dy) + ny * (z + dz));
                    const uint64_t a = rank[v], b = rank[w];
                    keys.push_back(a > b ? (a << 32) | b : (b << 32) | a);
                }
            }
    std::sort(keys.begin(), keys.end());
    /* union-find over ranks; the root of a component is its oldest (lowest) rank */
    std::vector<uint32_t> parent((size_t)V);
    for (int64_t i = 0; i < V; ++i) parent[(size_t)i] = (uint32_t)i;
    auto find = [&](uint32_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    };
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (uint64_t k : keys) {
        const uint32_t hi = (uint32_t)(k >> 32), lo = (uint32_t)k;
        uint32_t ra = find(hi), rb = find(lo);
        if (ra == rb) continue;
        const uint32_t young = ra > rb ? ra : rb, old = ra > rb ? rb : ra;
        parent[young] = old;
        if (young != hi) pairs.push_back({young, hi});  /* death at the edge's top vertex */
    }
    std::sort(pairs.begin(), pairs.end());
    for (size_t i = 0; i < pairs.size() && (int64_t)i < cap; ++i) {
        out[2 * i] = pairs[i].first;
        out[2 * i + 1] = pairs[i].second;
    }
    return (int64_t)pairs.size();
}

}  // extern "C"

extern "C" {

/* Persistent 1-cycle generators against their definition (Sec. 8): for a
 * D1 pair (tau, sigma), a representative is a 1-cycle z, homologous to the
 * boundary of sigma, that is born at tau. Over the lexicographic filtration
 * (simplices enumerated from the tetrahedra as above) that means:
 *   - z is a cycle: every vertex lies on an even number of its edges;
 *   - the highest edge of z is tau;
 *   - z + boundary(sigma) is a sum of boundaries of triangles that come
 *     before sigma (Z2 elimination over the triangles in filtration order).
 * Pairs and edges are given by vertex ids: pair i has birth edge
 * (tv[2i], tv[2i+1]) and death triangle (sv[3i..3i+2]); its cycle is the
 * edges ev[2k], ev[2k+1] for off[i] <= k < off[i+1]. status[i] = 0 when all
 * holds, 1 not a cycle, 2 an edge or simplex not in the complex, 3 highest
 * edge is not tau, 4 not homologous to boundary(sigma) before sigma. */
void bf_check_cycles(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t n, const int64_t* tv,
                     const int64_t* sv, const int64_t* off, const int64_t* ev, int32_t* status) {
    Complex K;
    all_simplices(nx, ny, nz, K);
    const size_t ns = K.simp.size();
    std::map<Verts, int> index;
    for (size_t i = 0; i < ns; ++i) index[K.simp[i]] = (int)i;
    std::vector<int> tri;  /* triangles in filtration order */
    for (size_t i = 0; i < ns; ++i)
        if (K.dim[i] == 2) tri.push_back((int)i);
    std::vector<std::array<i64, 4>> key(ns);
    for (size_t i = 0; i < ns; ++i) key[i] = lex_key(K.simp[i], rank);
    std::sort(tri.begin(), tri.end(), [&](int a, int b) { return key[a] < key[b]; });
    /* rows: edges by filtration position */
    std::vector<int> edges;
    for (size_t i = 0; i < ns; ++i)
        if (K.dim[i] == 1) edges.push_back((int)i);
    std::sort(edges.begin(), edges.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<int> row(ns, -1);
    for (size_t r = 0; r < edges.size(); ++r) row[edges[r]] = (int)r;
    auto find = [&](std::initializer_list<i64> vs) {
        Verts v = {-1, -1, -1, -1};
        int k = 0;
        for (i64 x : vs) v[k++] = x;
        std::sort(v.begin(), v.begin() + k);
        auto it = index.find(v);
        return it == index.end() ? -1 : it->second;
    };
    auto boundary = [&](int t) {
        std::vector<int> b;
        const Verts& v = K.simp[t];
        b.push_back(row[find({v[0], v[1]})]);
        b.push_back(row[find({v[0], v[2]})]);
        b.push_back(row[find({v[1], v[2]})]);
        std::sort(b.begin(), b.end());
        return b;
    };
    /* pairs by death triangle */
    std::map<int, std::vector<int64_t>> at;
    for (int64_t i = 0; i < n; ++i) {
        status[i] = 0;
        const int s = find({sv[3 * i], sv[3 * i + 1], sv[3 * i + 2]});
        const int t = find({tv[2 * i], tv[2 * i + 1]});
        if (s < 0 || t < 0 || K.dim[s] != 2 || K.dim[t] != 1) { status[i] = 2; continue; }
        std::vector<int> deg;
        std::vector<int> z;
        for (int64_t k = off[i]; k < off[i + 1]; ++k) {
            const int e = find({ev[2 * k], ev[2 * k + 1]});
            if (e < 0 || K.dim[e] != 1) { status[i] = 2; break; }
            z.push_back(row[e]);
            deg.push_back((int)ev[2 * k]);
            deg.push_back((int)ev[2 * k + 1]);
        }
        if (status[i]) continue;
        std::sort(deg.begin(), deg.end());
        for (size_t a = 0; a < deg.size();) {
            size_t b = a;
            while (b < deg.size() && deg[b] == deg[a]) ++b;
            if ((b - a) & 1) status[i] = 1;
            a = b;
        }
        if (status[i]) continue;
        std::sort(z.begin(), z.end());
        if (std::adjacent_find(z.begin(), z.end()) != z.end()) { status[i] = 1; continue; }
        if (z.empty() || z.back() != row[t]) { status[i] = 3; continue; }
        at[s].push_back(i);
        (void)z;
    }
    /* eliminate in filtration order; test each pair just before its sigma */
    std::vector<std::vector<int>> basis;
    std::vector<int> owner(edges.size(), -1);
    std::vector<int> tmp;
    auto reduce = [&](std::vector<int>& c) {
        while (!c.empty() && owner[c.back()] >= 0) sym_diff(c, basis[owner[c.back()]], tmp);
    };
    for (int s : tri) {
        std::vector<int> bs = boundary(s);
        auto it = at.find(s);
        if (it != at.end()) {
            for (int64_t i : it->second) {
                std::vector<int> z;
                for (int64_t k = off[i]; k < off[i + 1]; ++k) z.push_back(row[find({ev[2 * k], ev[2 * k + 1]})]);
                std::sort(z.begin(), z.end());
                sym_diff(z, bs, tmp);
                reduce(z);
                if (!z.empty()) status[i] = 4;
            }
        }
        reduce(bs);
        if (!bs.empty()) {
            owner[bs.back()] = (int)basis.size();
            basis.push_back(bs);
        }
    }
}

}  // extern "C"

extern "C" {

/* D2 in vertex-order space from the dual union-find over the whole
 * triangulation (Sec. 5.2, the dual of the Sec. 5.1 argument; PairSimplices
 * restricted to the top dimension, Sec. 2.5): every triangle, in decreasing
 * lexicographic order, joins the components of its two cofacet tetrahedra,
 * or of its one tetrahedron and the outside when it lies on the boundary of
 * the grid. A component is as old as its highest tetrahedron; the outside is
 * older than all. When two components meet, the younger one is filled: the
 * pair is (triangle, that component's highest tetrahedron). Triangles and
 * their cofacets are found from vertex coordinates (two vertices are joined
 * when their coordinates differ by a non-zero vector whose non-zero
 * components are all +1 or all -1; any 3 or 4 pairwise joined vertices span
 * a simplex), not from any id table. Output: (birth rank, death rank) of
 * every pair with positive persistence, sorted; returns their number. */
int64_t bf_d2_dual(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t* out, int64_t cap) {
    const int64_t V = nx * ny * nz;
    std::vector<uint32_t> order((size_t)V);
    for (int64_t v = 0; v < V; ++v) order[rank[v]] = (uint32_t)v;
    int nb[14][3];
    int nn = 0;
    for (int m = 1; m < 8; ++m)
        for (int sg = 1; sg >= -1; sg -= 2) {
            nb[nn][0] = sg * (m & 1);
            nb[nn][1] = sg * ((m >> 1) & 1);
            nb[nn][2] = sg * ((m >> 2) & 1);
            ++nn;
        }
    auto joined = [](const int* p, const int* q) {
        bool pos = true, neg = true, nzero = false;
        for (int a = 0; a < 3; ++a) {
            const int d = q[a] - p[a];
            if (d != 0 && d != 1) pos = false;
            if (d != 0 && d != -1) neg = false;
            if (d != 0) nzero = true;
        }
        return nzero && (pos || neg);
    };
    const int zero[3] = {0, 0, 0};
    /* a tetrahedron = (lowest corner, order in which its chain takes the
     * three axes): node anchor * 6 + code; from four corner offsets around
     * the vertex, the anchor offset and the code */
    auto tet_of = [&](const int pts[4][3], int anchor_off[3]) {
        int idx[4] = {0, 1, 2, 3};
        std::sort(idx, idx + 4, [&](int i, int j) {
            return pts[i][0] + pts[i][1] + pts[i][2] < pts[j][0] + pts[j][1] + pts[j][2];
        });
        int axis[3] = {0, 0, 0};
        for (int s = 0; s < 3; ++s)
            for (int a = 0; a < 3; ++a)
                if (pts[idx[s + 1]][a] != pts[idx[s]][a]) axis[s] = a;
        for (int a = 0; a < 3; ++a) anchor_off[a] = pts[idx[0]][a];
        return axis[0] * 2 + (axis[1] < axis[2] ? 0 : 1);
    };
    /* tables over the 14 neighbour offsets, derived from coordinates once:
     * which pairs are joined, and for a joined pair (a, b) the (at most two)
     * offsets c joined to 0, a and b, with the tetrahedron {0, a, b, c} */
    bool J[14][14];
    int ncof[14][14];
    int cof[14][14][2], cof_code[14][14][2], cof_anchor[14][14][2][3];
    for (int a = 0; a < 14; ++a)
        for (int b = 0; b < 14; ++b) {
            J[a][b] = a != b && joined(nb[a], nb[b]);
            ncof[a][b] = 0;
        }
    for (int a = 0; a < 14; ++a)
        for (int b = 0; b < 14; ++b) {
            if (!J[a][b] || !joined(zero, nb[a]) || !joined(zero, nb[b])) continue;
            for (int c = 0; c < 14; ++c) {
                if (c == a || c == b || !J[c][a] || !J[c][b]) continue;
                const int k = ncof[a][b]++;
                cof[a][b][k] = c;
                const int pts[4][3] = {{0, 0, 0}, {nb[a][0], nb[a][1], nb[a][2]}, {nb[b][0], nb[b][1], nb[b][2]},
                                       {nb[c][0], nb[c][1], nb[c][2]}};
                cof_code[a][b][k] = tet_of(pts, cof_anchor[a][b][k]);
            }
        }
    const int64_t OUT = 6 * V;
    std::vector<uint32_t> parent((size_t)(OUT + 1));
    for (int64_t i = 0; i <= OUT; ++i) parent[(size_t)i] = (uint32_t)i;
    auto find = [&](uint32_t a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    };
    /* age of a node: the ranks of its vertices, decreasing (outside: above all) */
    auto age = [&](uint32_t node, std::array<i64, 4>& k) {
        if (node == (uint32_t)OUT) {
            k = {V, V, V, V};
            return;
        }
        const int64_t anchor = node / 6;
        const int code = (int)(node % 6);
        const int a0 = code / 2;
        const int r1 = (a0 + 1) % 3, r2 = (a0 + 2) % 3;
        const int lo = r1 < r2 ? r1 : r2, hi = r1 < r2 ? r2 : r1;
        const int axes[3] = {a0, code % 2 ? hi : lo, code % 2 ? lo : hi};
        int c[3] = {(int)(anchor % nx), (int)((anchor / nx) % ny), (int)(anchor / (nx * ny))};
        k[0] = rank[anchor];
        for (int s = 0; s < 3; ++s) {
            c[axes[s]] += 1;
            k[s + 1] = rank[c[0] + nx * (c[1] + ny * (int64_t)c[2])];
        }
        std::sort(k.begin(), k.end(), [](i64 a, i64 b) { return a > b; });
    };
    std::vector<std::pair<int64_t, int64_t>> pairs;
    struct Tri { i64 k1, k2; int a, b; };
    std::vector<Tri> tris;
    for (int64_t r = V - 1; r >= 0; --r) {
        const int64_t x = order[(size_t)r];
        const int cx[3] = {(int)(x % nx), (int)((x / nx) % ny), (int)(x / (nx * ny))};
        bool in[14], lower[14];
        i64 rk[14];
        for (int n = 0; n < 14; ++n) {
            const int q[3] = {cx[0] + nb[n][0], cx[1] + nb[n][1], cx[2] + nb[n][2]};
            in[n] = q[0] >= 0 && q[1] >= 0 && q[2] >= 0 && q[0] < nx && q[1] < ny && q[2] < nz;
            rk[n] = in[n] ? rank[q[0] + nx * (q[1] + ny * (int64_t)q[2])] : -1;
            lower[n] = in[n] && rk[n] < r;
        }
        tris.clear();
        for (int i = 0; i < 14; ++i)
            for (int j = i + 1; j < 14; ++j)
                if (lower[i] && lower[j] && J[i][j])
                    tris.push_back({rk[i] > rk[j] ? rk[i] : rk[j], rk[i] > rk[j] ? rk[j] : rk[i], i, j});
        std::sort(tris.begin(), tris.end(), [](const Tri& u, const Tri& w) {
            return u.k1 != w.k1 ? u.k1 > w.k1 : u.k2 > w.k2;
        });
        for (const Tri& t : tris) {
            uint32_t side[2] = {(uint32_t)OUT, (uint32_t)OUT};
            int ns = 0;
            for (int k = 0; k < ncof[t.a][t.b]; ++k) {
                if (!in[cof[t.a][t.b][k]]) continue;
                const int* ao = cof_anchor[t.a][t.b][k];
                const int64_t anchor = (cx[0] + ao[0]) + nx * ((cx[1] + ao[1]) + ny * (int64_t)(cx[2] + ao[2]));
                side[ns++] = (uint32_t)(anchor * 6 + cof_code[t.a][t.b][k]);
            }
            const uint32_t ra = find(side[0]), rb = find(side[1]);
            if (ra == rb) continue;
            std::array<i64, 4> ka, kb;
            age(ra, ka);
            age(rb, kb);
            const bool a_young = ka < kb;
            const uint32_t young = a_young ? ra : rb, old = a_young ? rb : ra;
            const i64 death = a_young ? ka[0] : kb[0];
            parent[young] = old;
            if (death != r) pairs.push_back({r, death});
        }
    }
    std::sort(pairs.begin(), pairs.end());
    for (size_t i = 0; i < pairs.size() && (int64_t)i < cap; ++i) {
        out[2 * i] = pairs[i].first;
        out[2 * i + 1] = pairs[i].second;
    }
    return (int64_t)pairs.size();
}

}  // extern "C"
