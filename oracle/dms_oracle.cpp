/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential, deliberately unoptimised implementation of the
 * Discrete Morse Sandwich pipeline (Guillou, Vidal, Tierny) on a 3D regular
 * grid with the implicit 6-tetrahedra Freudenthal (Kuhn) triangulation.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. It shares no code, header or table with the GPU
 * library: every table below is written out independently here.
 *
 * Steps, in the paper's order:
 *   1. vertex order with a symbolic-perturbation tie break   (Sec. 2.1)
 *   2. lexicographic simplex order                            (Sec. 2.2)
 *   3. discrete gradient by expansions, ProcessLowerStars     (Sec. 2.6; Alg. "Zero-persistence skip")
 *   4. critical simplices, sorted by the lexicographic order  (Alg. "Zero-persistence skip")
 *   5. D0 from unstable sets of 1-saddles + union-find        (Sec. 5.1)
 *   6. D2 from stable sets of 2-saddles + dual union-find,
 *      with the virtual maximum for the domain boundary       (Sec. 5.2)
 *   7. D1 by PairCriticalSimplices on the unpaired 2-saddles  (Sec. 4, Alg. "PairCriticalSimplices")
 *   8. classes of infinite persistence                        (Sec. 6)
 * A grid with nz = 1 is a 2D grid (the plane z = 0 of the same
 * triangulation): there D1 comes from the dual union-find of step 6 applied
 * to the 1-saddles and triangles, and steps 6 (in 3D form) and 7 are skipped
 * (Sec. 3: the sandwich is needed for 3D data only).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - vertex id v = x + nx*(y + ny*z); ties of f broken by the lower vertex id;
 *     -0 == +0; NaN is rejected.
 *   - simplex id = anchor * T_k + type, anchor = the vertex with the smallest
 *     coordinates, T = {1, 7, 12, 6}; type tables below.
 *   - ProcessLowerStars follows Robins et al.: both queues are ordered sets
 *     keyed by the lexicographic order; a cell popped from the "one unpaired
 *     face" queue that was classified meanwhile is skipped.
 *   - the virtual maximum is on (exact diagram on a domain with boundary).
 */
#include <algorithm>
#include <omp.h>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

namespace {

typedef int64_t i64;

/* ---------------------------------------------------------------- grid -- */

struct Grid {
    i64 n[3];
    i64 V() const { return n[0] * n[1] * n[2]; }
    void xyz(i64 v, i64 c[3]) const {
        c[0] = v % n[0];
        c[1] = (v / n[0]) % n[1];
        c[2] = v / (n[0] * n[1]);
    }
    i64 vid(const i64 c[3]) const { return c[0] + n[0] * (c[1] + n[1] * c[2]); }
};

/* An axis set is a 3-bit mask: bit 0 = x, bit 1 = y, bit 2 = z. Every
 * simplex of the Kuhn triangulation is a chain w0 < w1 < ... < wk in one unit
 * cube whose successive steps are non-empty, pairwise disjoint axis sets. */
const int NTYPES[4] = {1, 7, 12, 6};
const int EDGE_STEP[7] = {1, 2, 3, 4, 5, 6, 7};
const int TRI_STEP[12][2] = {{1, 2}, {1, 4}, {1, 6}, {2, 1}, {2, 4}, {2, 5},
                             {3, 4}, {4, 1}, {4, 2}, {4, 3}, {5, 2}, {6, 1}};
const int TET_STEP[6][3] = {{1, 2, 4}, {1, 4, 2}, {2, 1, 4},
                            {2, 4, 1}, {4, 1, 2}, {4, 2, 1}};

int steps_of(int dim, int type, int out[3]) {
    if (dim == 1) { out[0] = EDGE_STEP[type]; return 1; }
    if (dim == 2) { out[0] = TRI_STEP[type][0]; out[1] = TRI_STEP[type][1]; return 2; }
    if (dim == 3) { for (int i = 0; i < 3; ++i) out[i] = TET_STEP[type][i]; return 3; }
    return 0;
}

void add_mask(i64 c[3], int mask, int sign) {
    for (int a = 0; a < 3; ++a)
        if (mask & (1 << a)) c[a] += sign;
}

/* Vertices of simplex (dim, id) in chain order; false if it is not in the grid. */
bool simplex_vertices(const Grid& g, int dim, i64 id, i64 out[4]) {
    if (id < 0) return false;
    i64 anchor = id / NTYPES[dim];
    int type = (int)(id % NTYPES[dim]);
    if (anchor >= g.V()) return false;
    int st[3];
    int ns = steps_of(dim, type, st);
    i64 c[3];
    g.xyz(anchor, c);
    out[0] = anchor;
    for (int s = 0; s < ns; ++s) {
        add_mask(c, st[s], +1);
        for (int a = 0; a < 3; ++a)
            if (c[a] >= g.n[a]) return false;
        out[s + 1] = g.vid(c);
    }
    return true;
}

/* Inverse of simplex_vertices: a sorted vertex chain -> (dim, id), or -1. */
i64 simplex_from_vertices(const Grid& g, int dim, const i64* vs) {
    if (dim == 0) return vs[0];
    int st[3];
    i64 c0[3], c1[3];
    for (int s = 0; s < dim; ++s) {
        g.xyz(vs[s], c0);
        g.xyz(vs[s + 1], c1);
        int m = 0;
        for (int a = 0; a < 3; ++a) {
            i64 d = c1[a] - c0[a];
            if (d == 1) m |= 1 << a;
            else if (d != 0) return -1;
        }
        if (m == 0) return -1;
        st[s] = m;
    }
    for (int t = 0; t < NTYPES[dim]; ++t) {
        int ref[3];
        steps_of(dim, t, ref);
        bool ok = true;
        for (int s = 0; s < dim; ++s) ok = ok && (ref[s] == st[s]);
        if (ok) return vs[0] * NTYPES[dim] + t;
    }
    return -1;
}

/* All simplices of dimension >= 1 that contain vertex x: x sits at some
 * position p of the chain, so the anchor is x minus the first p steps. */
void star_of(const Grid& g, i64 x, std::vector<std::pair<int, i64>>& out) {
    out.clear();
    i64 cx[3];
    g.xyz(x, cx);
    for (int dim = 1; dim <= 3; ++dim) {
        for (int t = 0; t < NTYPES[dim]; ++t) {
            int st[3];
            steps_of(dim, t, st);
            for (int p = 0; p <= dim; ++p) {
                i64 c[3] = {cx[0], cx[1], cx[2]};
                bool ok = true;
                for (int s = 0; s < p; ++s) add_mask(c, st[s], -1);
                for (int a = 0; a < 3; ++a) ok = ok && c[a] >= 0;
                if (!ok) continue;
                i64 id = g.vid(c) * NTYPES[dim] + t;
                i64 vs[4];
                if (simplex_vertices(g, dim, id, vs)) out.push_back({dim, id});
            }
        }
    }
}

/* ------------------------------------------------------- vertex order -- */

/* Sec. 2.1: f is made injective by a symbolic perturbation. Reading: order
 * by (f, vertex id) with -0 == +0; NaN has no place in a total order. */
bool vertex_order(const float* f, i64 V, std::vector<uint32_t>& rank) {
    std::vector<i64> idx(V);
    for (i64 v = 0; v < V; ++v) {
        if (std::isnan(f[v])) return false;
        idx[v] = v;
    }
    std::stable_sort(idx.begin(), idx.end(), [&](i64 a, i64 b) {
        float fa = f[a] == 0.0f ? 0.0f : f[a];
        float fb = f[b] == 0.0f ? 0.0f : f[b];
        return fa < fb;
    });
    rank.assign(V, 0);
    for (i64 i = 0; i < V; ++i) rank[idx[i]] = (uint32_t)i;
    return true;
}

/* ------------------------------------------------- lexicographic order -- */

/* Sec. 2.2: compare the vertex values sorted in decreasing order, element by
 * element; a face (a proper prefix) is smaller than its cofaces. Padding
 * with -1 realises the prefix rule since every rank is >= 0. */
struct Key {
    i64 r[4];
    bool operator<(const Key& o) const {
        for (int i = 0; i < 4; ++i)
            if (r[i] != o.r[i]) return r[i] < o.r[i];
        return false;
    }
    bool operator==(const Key& o) const {
        for (int i = 0; i < 4; ++i)
            if (r[i] != o.r[i]) return false;
        return true;
    }
};

struct Ctx;

/* ------------------------------------------------------------- state -- */

struct Ctx {
    Grid g;
    std::vector<uint32_t> rank;
    /* Discrete gradient: partner[dim][id] = partner_id * 4 + partner_dim,
     * -1 for a critical simplex, -2 for an id outside the grid. */
    std::vector<i64> partner[4];
    std::vector<i64> crit[4];              /* sorted ascending by Key */
    std::vector<i64> d0, d1, d2;           /* flattened (birth, death) */
    std::vector<i64> arcs0, arcs2;         /* flattened (node_a, node_b, saddle) */
    /* Sec. 8: the boundary cached when a 2-saddle was paired (its
     * persistent 1-cycle generator), by 2-saddle id */
    std::map<i64, std::vector<i64>> gen1;
    std::vector<i64> gen1_off, gen1_edges; /* per finite D1 pair, in output order */
    double times[6] = {0, 0, 0, 0, 0, 0};  /* order, gradient, sort, D0+D2, D1, total */
    i64 d1_adds = 0;                       /* D1 steps that added an earlier 2-saddle's boundary */
    std::string err;

    Key key(int dim, i64 id) const {
        i64 vs[4];
        simplex_vertices(g, dim, id, vs);
        Key k;
        for (int i = 0; i < 4; ++i) k.r[i] = -1;
        for (int i = 0; i <= dim; ++i) k.r[i] = rank[vs[i]];
        std::sort(k.r, k.r + dim + 1, [](i64 a, i64 b) { return a > b; });
        return k;
    }

    i64 max_vertex(int dim, i64 id) const {
        i64 vs[4];
        simplex_vertices(g, dim, id, vs);
        i64 best = vs[0];
        for (int i = 1; i <= dim; ++i)
            if (rank[vs[i]] > rank[best]) best = vs[i];
        return best;
    }

    /* facets: all vertex subsets of size dim, as simplex ids */
    void facets(int dim, i64 id, std::vector<i64>& out) const {
        out.clear();
        i64 vs[4];
        simplex_vertices(g, dim, id, vs);
        for (int drop = 0; drop <= dim; ++drop) {
            i64 sub[4];
            int k = 0;
            for (int i = 0; i <= dim; ++i)
                if (i != drop) sub[k++] = vs[i];
            out.push_back(simplex_from_vertices(g, dim - 1, sub));
        }
    }

    /* cofacets: the (dim+1)-simplices in the star of the first vertex that
     * contain every vertex of the simplex */
    void cofacets(int dim, i64 id, std::vector<i64>& out) const {
        out.clear();
        i64 vs[4];
        simplex_vertices(g, dim, id, vs);
        std::vector<std::pair<int, i64>> st;
        star_of(g, vs[0], st);
        for (auto& s : st) {
            if (s.first != dim + 1) continue;
            i64 ws[4];
            simplex_vertices(g, dim + 1, s.second, ws);
            int hit = 0;
            for (int i = 0; i <= dim; ++i)
                for (int j = 0; j <= dim + 1; ++j) hit += (vs[i] == ws[j]);
            if (hit == dim + 1) out.push_back(s.second);
        }
    }
};

/* ------------------------------------------------- ProcessLowerStars -- */

struct Cell {
    int dim;
    i64 id;
    i64 vs[4];
    Key key;
};

enum { UNCLASSIFIED = 0, PAIRED = 1, CRITICAL = 2 };

/* Discrete gradient of the lower star of x by expansions (Robins et al.,
 * used by the paper in Sec. 2.6 and Alg. "Zero-persistence skip"). The lower
 * star holds the simplices whose highest vertex is x. Faces and cofaces
 * below are the facets / cofacets that also lie in the lower star. */
void process_lower_star(Ctx& C, i64 x, std::vector<std::pair<int, i64>>& star,
                        std::vector<std::pair<i64, i64>>* pairs_out = nullptr,
                        std::vector<i64>* crit_out = nullptr) {
    const Grid& g = C.g;
    std::vector<Cell> L;
    Cell cx;
    cx.dim = 0;
    cx.id = x;
    cx.vs[0] = x;
    cx.key = C.key(0, x);
    L.push_back(cx);
    star_of(g, x, star);
    for (auto& s : star) {
        Cell c;
        c.dim = s.first;
        c.id = s.second;
        simplex_vertices(g, c.dim, c.id, c.vs);
        bool lower = true;
        for (int i = 0; i <= c.dim; ++i)
            if (c.vs[i] != x && C.rank[c.vs[i]] > C.rank[x]) lower = false;
        if (!lower) continue;
        c.key = C.key(c.dim, c.id);
        L.push_back(c);
    }
    const int n = (int)L.size();
    std::vector<int> state(n, UNCLASSIFIED), mate(n, -1);
    auto record = [&](int a, int b) {  /* a is the tail, b the head */
        state[a] = state[b] = PAIRED;
        mate[a] = b;
        mate[b] = a;
    };
    if (n == 1) {
        state[0] = CRITICAL;
    } else {
        /* face / coface incidences inside the lower star, by vertex sets */
        std::vector<std::vector<int>> faces(n), cofaces(n);
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                if (L[b].dim != L[a].dim + 1) continue;
                int hit = 0;
                for (int i = 0; i <= L[a].dim; ++i)
                    for (int j = 0; j <= L[b].dim; ++j) hit += (L[a].vs[i] == L[b].vs[j]);
                if (hit == L[a].dim + 1) {
                    faces[b].push_back(a);
                    cofaces[a].push_back(b);
                }
            }
        auto unpaired = [&](int a) {
            int k = 0;
            for (int f : faces[a]) k += (state[f] == UNCLASSIFIED);
            return k;
        };
        typedef std::set<std::pair<Key, int>> PQ;
        PQ pq_zero, pq_one;
        /* x pairs with its lowest edge */
        int delta = -1;
        for (int a = 1; a < n; ++a)
            if (L[a].dim == 1 && (delta < 0 || L[a].key < L[delta].key)) delta = a;
        record(0, delta);
        for (int a = 1; a < n; ++a)
            if (L[a].dim == 1 && a != delta) pq_zero.insert({L[a].key, a});
        for (int b : cofaces[delta])
            if (unpaired(b) == 1) pq_one.insert({L[b].key, b});
        while (!pq_one.empty() || !pq_zero.empty()) {
            while (!pq_one.empty()) {
                int a = pq_one.begin()->second;
                pq_one.erase(pq_one.begin());
                if (state[a] != UNCLASSIFIED) continue;
                if (unpaired(a) == 0) {
                    pq_zero.insert({L[a].key, a});
                    continue;
                }
                int p = -1;
                for (int f : faces[a])
                    if (state[f] == UNCLASSIFIED) p = f;
                record(p, a);
                pq_zero.erase({L[p].key, p});
                for (int b : cofaces[a])
                    if (unpaired(b) == 1) pq_one.insert({L[b].key, b});
                for (int b : cofaces[p])
                    if (unpaired(b) == 1) pq_one.insert({L[b].key, b});
            }
            if (!pq_zero.empty()) {
                int c = pq_zero.begin()->second;
                pq_zero.erase(pq_zero.begin());
                if (state[c] != UNCLASSIFIED) continue;
                state[c] = CRITICAL;
                for (int b : cofaces[c])
                    if (unpaired(b) == 1) pq_one.insert({L[b].key, b});
            }
        }
    }
    for (int a = 0; a < n; ++a) {
        if (state[a] == UNCLASSIFIED) throw std::runtime_error("lower star left a cell unclassified");
        i64 code = state[a] == CRITICAL ? -1 : L[mate[a]].id * 4 + L[mate[a]].dim;
        if (pairs_out) pairs_out->push_back({L[a].id * 4 + L[a].dim, code});
        else C.partner[L[a].dim][L[a].id] = code;
        if (crit_out && state[a] == CRITICAL) crit_out->push_back(L[a].id * 4 + L[a].dim);
    }
}

void gradient(Ctx& C) {
    const i64 V = C.g.V();
    for (int d = 0; d < 4; ++d) C.partner[d].assign(V * NTYPES[d], -2);
    std::vector<std::pair<int, i64>> star;
    for (i64 x = 0; x < V; ++x) process_lower_star(C, x, star);
}

/* --------------------------------------------------- critical simplices -- */

/* Alg. "Zero-persistence skip": unpaired simplices form C_k, sorted by the
 * lexicographic order. */
void critical_sets(Ctx& C) {
    for (int d = 0; d < 4; ++d) {
        std::vector<std::pair<Key, i64>> tmp;
        const std::vector<i64>& P = C.partner[d];
        for (i64 id = 0; id < (i64)P.size(); ++id)
            if (P[id] == -1) tmp.push_back({C.key(d, id), id});
        std::sort(tmp.begin(), tmp.end());
        C.crit[d].clear();
        for (auto& t : tmp) C.crit[d].push_back(t.second);
    }
}

/* ------------------------------------------------------------------ D0 -- */

struct UF {
    std::unordered_map<i64, i64> parent;
    i64 find(i64 a) {
        auto it = parent.find(a);
        if (it == parent.end()) return a;
        i64 r = find(it->second);
        it->second = r;
        return r;
    }
};

/* Sec. 5.1: the unstable set of a critical edge is its two descending
 * v-paths; each regular vertex continues through its paired edge to the
 * edge's other vertex until a minimum. The arcs are then merged in
 * increasing order; the younger (higher) root dies and the older one stays
 * the representative. */
void diagram0(Ctx& C, std::vector<char>& edge_paired, std::vector<char>& min_paired) {
    const Grid& g = C.g;
    auto descend = [&](i64 v) {
        for (;;) {
            i64 p = C.partner[0][v];
            if (p == -1) return v;
            i64 vs[4];
            simplex_vertices(g, 1, p / 4, vs);
            v = (vs[0] == v) ? vs[1] : vs[0];
        }
    };
    UF uf;
    const std::vector<i64>& C1 = C.crit[1];
    edge_paired.assign(C1.size(), 0);
    for (size_t k = 0; k < C1.size(); ++k) {
        i64 vs[4];
        simplex_vertices(g, 1, C1[k], vs);
        i64 ma = descend(vs[0]), mb = descend(vs[1]);
        C.arcs0.push_back(ma);
        C.arcs0.push_back(mb);
        C.arcs0.push_back(C1[k]);
        i64 ra = uf.find(ma), rb = uf.find(mb);
        if (ra == rb) continue;
        i64 young = C.rank[ra] > C.rank[rb] ? ra : rb;
        i64 old = young == ra ? rb : ra;
        C.d0.push_back(young);
        C.d0.push_back(C1[k]);
        uf.parent[young] = old;
        edge_paired[k] = 1;
    }
    min_paired.assign(C.crit[0].size(), 0);
    std::unordered_map<i64, size_t> at;
    for (size_t k = 0; k < C.crit[0].size(); ++k) at[C.crit[0][k]] = k;
    for (size_t k = 0; k < C.d0.size(); k += 2) min_paired[at[C.d0[k]]] = 1;
}

/* ------------------------------------------------------------------ D2 -- */

/* Sec. 5.2: by duality the stable set of a critical (n-1)-saddle, n the
 * dimension of the grid's top simplices, is followed through n-simplices:
 * enter a cofacet; while it is regular, leave through its paired facet into
 * the n-simplex on the other side. Leaving the domain reaches the virtual
 * maximum (value +infinity, the outside). Arcs are merged in decreasing
 * order; the younger root is the lower n-simplex. On a 3D grid this is D2
 * over the 2-saddles (triangles into tetrahedra); on a 2D grid it is D1 over
 * the 1-saddles (edges into triangles), where no sandwich is needed (Sec. 3). */
const i64 VIRTUAL = -1;

/* virtual_max = false: the optional adjustment of Sec. 5.2 is off -- the
 * outside is no node: an arc that reaches it joins nothing, and its saddle
 * stays unpaired here. */
/* skip (optional, virtual maximum off): saddles to leave out, by position in
 * C.crit[d] -- on a 2D grid the 1-saddles D0 already paired: with the
 * virtual maximum they join two triangles of one component anyway (so the
 * rule leaves them out by itself), without it they could join two, and a
 * saddle is the birth or the death of one class only. */
void diagram_dual(Ctx& C, int d, std::vector<char>& saddle_paired, std::vector<i64>& pairs, bool virtual_max = true,
                  const std::vector<char>* skip = nullptr) {
    const int top = d + 1;
    std::vector<i64> cof;
    auto other_side = [&](i64 facet, i64 cell) {
        C.cofacets(d, facet, cof);
        for (i64 t : cof)
            if (t != cell) return t;
        return VIRTUAL;
    };
    auto ascend = [&](i64 cell) {
        while (cell != VIRTUAL) {
            i64 p = C.partner[top][cell];
            if (p == -1) return cell;
            cell = other_side(p / 4, cell);
        }
        return VIRTUAL;
    };
    UF uf;
    const std::vector<i64>& S = C.crit[d];
    saddle_paired.assign(S.size(), 0);
    for (size_t kk = S.size(); kk-- > 0;) {
        i64 t = S[kk];
        C.cofacets(d, t, cof);
        i64 side[2] = {VIRTUAL, VIRTUAL};
        for (size_t s = 0; s < cof.size() && s < 2; ++s) side[s] = cof[s];
        i64 ma = ascend(side[0]), mb = ascend(side[1]);
        C.arcs2.push_back(ma);
        C.arcs2.push_back(mb);
        C.arcs2.push_back(t);
        if (!virtual_max && (ma == VIRTUAL || mb == VIRTUAL)) continue;
        if (skip && (*skip)[kk]) continue;
        i64 ra = uf.find(ma), rb = uf.find(mb);
        if (ra == rb) continue;
        i64 young;
        if (ra == VIRTUAL) young = rb;
        else if (rb == VIRTUAL) young = ra;
        else young = C.key(top, ra) < C.key(top, rb) ? ra : rb;
        i64 old = young == ra ? rb : ra;
        pairs.push_back(t);
        pairs.push_back(young);
        uf.parent[young] = old;
        saddle_paired[kk] = 1;
    }
}

/* ------------------------------------------------------------------ D1 -- */

/* Sec. 4 with the sandwich of Sec. 3: the critical triangles left unpaired
 * by D2 are processed in increasing order. The boundary is kept as a set of
 * edges (mod-2 sums toggle membership). The highest edge tau decides:
 * a critical edge with no partner yet pairs with the triangle; a critical
 * edge already paired with an earlier triangle adds that triangle's cached
 * boundary; a regular edge adds the boundary of its gradient partner. */
/* sandwich = false: the ablation without the sandwich (Sec. 3): every
 * critical triangle is processed, and one whose boundary reduces to zero
 * (a triangle D2 pairs with a tetrahedron) is skipped. */
/* virtual_max = false: D2 left unpaired the 2-saddles whose arcs reached
 * the outside; those that create a 2-cycle reduce to zero here and stay
 * unpaired (classes of infinite persistence, Sec. 6). */
/* cache = false: the ablation without boundary caching (Sec. 4.1(b)); when
 * the top is the pivot of an earlier 2-saddle, that 2-saddle's own boundary
 * is added and reduced again instead of its cached reduced boundary. */
void diagram1(Ctx& C, const std::vector<char>& edge_paired0, const std::vector<char>& tri_paired2,
              bool sandwich = true, bool virtual_max = true, bool cache = true) {
    typedef std::pair<std::pair<i64, i64>, i64> EK;  /* ((rank max, rank min), edge id) */
    auto ekey = [&](i64 e) {
        Key k = C.key(1, e);
        return EK({k.r[0], k.r[1]}, e);
    };
    std::unordered_map<i64, size_t> crit_edge_at;
    for (size_t k = 0; k < C.crit[1].size(); ++k) crit_edge_at[C.crit[1][k]] = k;
    std::unordered_map<i64, i64> edge_owner;               /* critical edge -> triangle */
    std::unordered_map<i64, std::vector<i64>> cached;      /* triangle -> boundary edges */
    std::vector<i64> fs;
    const std::vector<i64>& C2 = C.crit[2];
    for (size_t kk = 0; kk < C2.size(); ++kk) {
        if (sandwich && tri_paired2[kk]) continue;
        i64 sigma = C2[kk];
        std::set<EK> B;
        auto toggle = [&](i64 e) {
            EK k = ekey(e);
            auto it = B.find(k);
            if (it == B.end()) B.insert(k);
            else B.erase(it);
        };
        C.facets(2, sigma, fs);
        for (i64 e : fs) toggle(e);
        i64 guard = 0;
        for (;;) {
            if (B.empty()) {
                if (sandwich && virtual_max) throw std::runtime_error("D1: boundary vanished on an unpaired 2-saddle");
                break;  /* a positive triangle: no D1 pair */
            }
            if (++guard > (i64)4e9) throw std::runtime_error("D1: no progress");
            i64 tau = B.rbegin()->second;
            i64 p = C.partner[1][tau];
            if (p == -1) {
                size_t at = crit_edge_at.at(tau);
                if (edge_paired0[at]) throw std::runtime_error("D1: a D0-paired edge became a pivot");
                auto ow = edge_owner.find(tau);
                if (ow == edge_owner.end()) {
                    edge_owner[tau] = sigma;
                    std::vector<i64>& cb = cached[sigma];
                    for (auto& k : B) cb.push_back(k.second);
                    C.gen1[sigma] = cb;
                    C.d1.push_back(tau);
                    C.d1.push_back(sigma);
                    break;
                }
                if (cache) {
                    for (i64 e : cached.at(ow->second)) toggle(e);
                } else {
                    C.facets(2, ow->second, fs);
                    for (i64 e : fs) toggle(e);
                }
                ++C.d1_adds;
            } else {
                if ((p & 3) != 2) throw std::runtime_error("D1: pivot edge is paired with a vertex");
                C.facets(2, p / 4, fs);
                for (i64 e : fs) toggle(e);
            }
        }
    }
}

/* ------------------------------------------------------------ pipeline -- */

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void sort_pairs(std::vector<i64>& p) {
    std::vector<std::pair<i64, i64>> t;
    for (size_t i = 0; i < p.size(); i += 2) t.push_back({p[i], p[i + 1]});
    std::sort(t.begin(), t.end(), [](const std::pair<i64, i64>& a, const std::pair<i64, i64>& b) {
        bool ea = a.second < 0, eb = b.second < 0;  /* essential classes last */
        if (ea != eb) return !ea;
        return a < b;
    });
    p.clear();
    for (auto& q : t) {
        p.push_back(q.first);
        p.push_back(q.second);
    }
}

void run(Ctx& C, const float* f, bool sandwich = true, bool virtual_max = true, bool cache = true) {
    double t0 = now();
    if (!vertex_order(f, C.g.V(), C.rank)) throw std::invalid_argument("NaN in the scalar field");
    double t1 = now();
    gradient(C);
    double t2 = now();
    critical_sets(C);
    double t3 = now();
    std::vector<char> e0, m0, t2p, e1p;
    const bool flat = C.g.n[2] == 1;  /* a 2D grid: the plane z = 0 */
    diagram0(C, e0, m0);
    if (flat) diagram_dual(C, 1, e1p, C.d1, virtual_max, virtual_max ? nullptr : &e0);
    else diagram_dual(C, 2, t2p, C.d2, virtual_max);
    double t4 = now();
    if (!flat) diagram1(C, e0, t2p, sandwich, virtual_max, cache);
    double t5 = now();
    /* Sec. 6: what stays unpaired is a class of infinite persistence */
    for (size_t k = 0; k < C.crit[0].size(); ++k)
        if (!m0[k]) { C.d0.push_back(C.crit[0][k]); C.d0.push_back(-1); }
    std::set<i64> used1, used2;
    for (size_t k = 1; k < C.d0.size(); k += 2) if (C.d0[k] >= 0) used1.insert(C.d0[k]);
    for (size_t k = 0; k < C.d1.size(); k += 2) { used1.insert(C.d1[k]); used2.insert(C.d1[k + 1]); }
    for (size_t k = 0; k < C.d2.size(); k += 2) used2.insert(C.d2[k]);
    for (i64 e : C.crit[1]) if (!used1.count(e)) { C.d1.push_back(e); C.d1.push_back(-1); }
    for (i64 t : C.crit[2]) if (!used2.count(t)) { C.d2.push_back(t); C.d2.push_back(-1); }
    sort_pairs(C.d0);
    sort_pairs(C.d1);
    sort_pairs(C.d2);
    /* generators in the order of the finite D1 pairs, edge ids ascending
     * (3D only: on a 2D grid D1 comes from the dual union-find) */
    C.gen1_off.push_back(0);
    for (size_t k = 0; k < C.d1.size() && !flat; k += 2) {
        if (C.d1[k + 1] < 0) continue;
        std::vector<i64> z = C.gen1.at(C.d1[k + 1]);
        std::sort(z.begin(), z.end());
        C.gen1_edges.insert(C.gen1_edges.end(), z.begin(), z.end());
        C.gen1_off.push_back((i64)C.gen1_edges.size());
    }
    C.times[0] = t1 - t0;
    C.times[1] = t2 - t1;
    C.times[2] = t3 - t2;
    C.times[3] = t4 - t3;
    C.times[4] = t5 - t4;
    C.times[5] = now() - t0;
}

}  // namespace

/* ------------------------------------------------------------- C API -- */

extern "C" {

enum {
    ORC_RANK = 0,          /* u32[V]                                   */
    ORC_PARTNER0 = 1,      /* i64[T_d * V] for d = 0..3 (1..4)         */
    ORC_CRIT0 = 5,         /* i64 sorted critical ids, d = 0..3 (5..8) */
    ORC_D0 = 9, ORC_D1 = 10, ORC_D2 = 11, /* i64 (birth, death) pairs  */
    ORC_ARCS0 = 12, ORC_ARCS2 = 13,       /* i64 (a, b, saddle)        */
    ORC_TIMES = 14,        /* f64[6]                                   */
    ORC_GEN1_OFF = 15,     /* i64 offsets of the D1 generators (n1 + 1) */
    ORC_GEN1_EDGES = 16,   /* i64 edge ids of the D1 generators         */
    ORC_D1_ADDS = 17       /* i64[1] additions of earlier boundaries in D1 */
};

/* flags bit 0: D1 without the sandwich (the ablation of Sec. 3);
 * bit 1: no virtual maximum on the domain boundary (Sec. 5.2, App. A) */
int orc_run_opts(int64_t nx, int64_t ny, int64_t nz, const float* f, int flags, void** out, char* err,
                 int errlen) {
    Ctx* C = new Ctx();
    C->g.n[0] = nx; C->g.n[1] = ny; C->g.n[2] = nz;
    try {
        if (nx < 2 || ny < 2 || nz < 1)
            throw std::invalid_argument("nx and ny must be >= 2, nz >= 1 (nz = 1: a 2D grid)");
        /* the ablation without the sandwich (Sec. 3) equals the sandwich only
         * when D2 is the plain reduction's, i.e. with the virtual maximum */
        if ((flags & 1) && (flags & 2))
            throw std::invalid_argument("the ablation without the sandwich needs the virtual maximum");
        run(*C, f, !(flags & 1), !(flags & 2), !(flags & 4));
    } catch (const std::exception& e) {
        if (err && errlen > 0) { std::strncpy(err, e.what(), errlen - 1); err[errlen - 1] = 0; }
        delete C;
        *out = nullptr;
        return -1;
    }
    *out = C;
    return 0;
}

int orc_run(int64_t nx, int64_t ny, int64_t nz, const float* f, void** out, char* err, int errlen) {
    return orc_run_opts(nx, ny, nz, f, 0, out, err, errlen);
}

int64_t orc_size(void* h, int what) {
    Ctx* C = (Ctx*)h;
    switch (what) {
        case ORC_RANK: return (int64_t)C->rank.size();
        case 1: case 2: case 3: case 4: return (int64_t)C->partner[what - 1].size();
        case 5: case 6: case 7: case 8: return (int64_t)C->crit[what - 5].size();
        case ORC_D0: return (int64_t)C->d0.size() / 2;
        case ORC_D1: return (int64_t)C->d1.size() / 2;
        case ORC_D2: return (int64_t)C->d2.size() / 2;
        case ORC_ARCS0: return (int64_t)C->arcs0.size() / 3;
        case ORC_ARCS2: return (int64_t)C->arcs2.size() / 3;
        case ORC_TIMES: return 6;
        case ORC_GEN1_OFF: return (int64_t)C->gen1_off.size();
        case ORC_GEN1_EDGES: return (int64_t)C->gen1_edges.size();
        case ORC_D1_ADDS: return 1;
    }
    return -1;
}

void orc_copy(void* h, int what, void* dst) {
    Ctx* C = (Ctx*)h;
    auto cp = [&](const std::vector<i64>& v) { std::memcpy(dst, v.data(), v.size() * sizeof(i64)); };
    switch (what) {
        case ORC_RANK: std::memcpy(dst, C->rank.data(), C->rank.size() * 4); break;
        case 1: case 2: case 3: case 4: cp(C->partner[what - 1]); break;
        case 5: case 6: case 7: case 8: cp(C->crit[what - 5]); break;
        case ORC_D0: cp(C->d0); break;
        case ORC_D1: cp(C->d1); break;
        case ORC_D2: cp(C->d2); break;
        case ORC_ARCS0: cp(C->arcs0); break;
        case ORC_ARCS2: cp(C->arcs2); break;
        case ORC_TIMES: std::memcpy(dst, C->times, sizeof(C->times)); break;
        case ORC_GEN1_OFF: cp(C->gen1_off); break;
        case ORC_GEN1_EDGES: cp(C->gen1_edges); break;
        case ORC_D1_ADDS: std::memcpy(dst, &C->d1_adds, sizeof(i64)); break;
    }
}

void orc_free(void* h) { delete (Ctx*)h; }

/* Vertex order only (Sec. 2.1). Returns -1 on NaN. */
int orc_vertex_order(int64_t V, const float* f, uint32_t* rank) {
    std::vector<uint32_t> r;
    if (!vertex_order(f, V, r)) return -1;
    std::memcpy(rank, r.data(), V * 4);
    return 0;
}

/* ProcessLowerStars on a sample of vertices only, for checks on grids too
 * large for the whole oracle. For each sampled vertex, writes up to 75
 * (cell, partner) records, cell = id*4+dim, partner = id*4+dim or -1;
 * unused records are (-2, -2). */
int orc_lower_star_sample(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t n,
                          const int64_t* verts, int64_t* out) {
    Ctx C;
    C.g.n[0] = nx; C.g.n[1] = ny; C.g.n[2] = nz;
    C.rank.assign(rank, rank + nx * ny * nz);
    std::vector<std::pair<int, i64>> star;
    std::vector<std::pair<i64, i64>> recs;
    try {
        for (int64_t s = 0; s < n; ++s) {
            recs.clear();
            process_lower_star(C, verts[s], star, &recs);
            for (int k = 0; k < 75; ++k) {
                out[(s * 75 + k) * 2 + 0] = k < (int)recs.size() ? recs[k].first : -2;
                out[(s * 75 + k) * 2 + 1] = k < (int)recs.size() ? recs[k].second : -2;
            }
        }
    } catch (const std::exception&) {
        return -1;
    }
    return 0;
}

/* Gradient of the whole grid from given ranks (ProcessLowerStars at every
 * vertex) -- used to time the gradient stage alone on a bounded sample. */
double orc_time_gradient(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t n_verts) {
    Ctx C;
    C.g.n[0] = nx; C.g.n[1] = ny; C.g.n[2] = nz;
    C.rank.assign(rank, rank + nx * ny * nz);
    for (int d = 0; d < 4; ++d) C.partner[d].assign(C.g.V() * NTYPES[d], -2);
    std::vector<std::pair<int, i64>> star;
    double t0 = now();
    for (i64 x = 0; x < n_verts && x < C.g.V(); ++x) process_lower_star(C, x, star);
    return now() - t0;
}

/* The same stage with the vertices shared among OpenMP threads: every cell
 * belongs to the lower star of exactly one vertex, so the lower stars are
 * independent (the paper parallelises this stage over vertices, Sec. 7.2).
 * *threads receives the number of threads that ran. */
double orc_time_gradient_omp(int64_t nx, int64_t ny, int64_t nz, const uint32_t* rank, int64_t n_verts,
                             int32_t* threads) {
    Ctx C;
    C.g.n[0] = nx; C.g.n[1] = ny; C.g.n[2] = nz;
    C.rank.assign(rank, rank + nx * ny * nz);
    for (int d = 0; d < 4; ++d) C.partner[d].assign(C.g.V() * NTYPES[d], -2);
    const i64 n = std::min<i64>(n_verts, C.g.V());
    int used = 1;
    double t0 = now();
#pragma omp parallel
    {
        std::vector<std::pair<int, i64>> star;
#pragma omp single
        used = omp_get_num_threads();
#pragma omp for schedule(dynamic, 4096)
        for (i64 x = 0; x < n; ++x) process_lower_star(C, x, star);
    }
    const double dt = now() - t0;
    if (threads) *threads = used;
    return dt;
}

}  // extern "C"
