"""Pins of the CPU oracle to things other than itself (CPU only).

* brute force: the full lexicographic filtration reduced column by column
  (PairSimplices is boundary-matrix reduction, Sec. 2.5), compared in
  vertex-order space after dropping zero-persistence pairs (Sec. 4.1(c));
  exhaustive over all 8! vertex orders of one cube, random on small grids;
* lower-link Betti numbers: the expansion-based gradient puts exactly
  b~_{k-1}(lower link) critical k-cells in each lower star (Sec. 1.1, 2.6);
* closed forms: simplex counts, Euler characteristic of the cube, the one
  essential class, hand-built fields with known extrema (elevation, Sec. 8.1);
* definitions: gradient pairs are facet/cofacet pairs inside one lower star,
  each simplex in at most one pair, and v-paths are acyclic (Sec. 2.6).
"""
import itertools

import numpy as np
import pytest

import oracle
import synthfields as sf
from tests import helpers as H


def _bf_equal(field):
    res = oracle.run(field)
    fin, ess = oracle.order_space(res)
    bp, be = oracle.bf_diagram(res.shape, res.rank)
    assert H.as_set(bp) == fin
    assert H.as_set(be) == ess
    return res


def _closed_counts(shape):
    nz, ny, nx = shape
    n = (nx, ny, nz)
    E = 0
    for d in itertools.product((0, 1), repeat=3):
        if sum(d) == 0:
            continue
        E += int(np.prod([n[a] - d[a] for a in range(3)]))
    cubes = (nx - 1) * (ny - 1) * (nz - 1)
    T = 2 * ((nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1)) + 6 * cubes
    return [nx * ny * nz, E, T, 6 * cubes]


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 3, 2), (2, 5, 3), (16, 16, 16), (7, 9, 11)])
def test_simplex_counts_closed_form(shape):
    assert list(oracle.bf_counts(shape)) == _closed_counts(shape)
    f = sf.noise(shape, 1)
    res = oracle.run(f)
    for d in range(4):
        assert int((res.partner[d] != -2).sum()) == _closed_counts(shape)[d]


def test_closed_form_values_at_16_and_512():
    # counts at 16^3 and 512^3 (the second is formula-only)
    assert _closed_counts((16, 16, 16)) == [4096, 25695, 41850, 20250]
    assert _closed_counts((512, 512, 512)) == [134217728, 936381439, 1602760698, 800596986]


def test_vertex_order_matches_stable_argsort_with_ties():
    rng = np.random.default_rng(3)
    f = rng.integers(0, 7, size=(5, 6, 7)).astype(np.float32)
    f.ravel()[::5] = -0.0
    f.ravel()[1::11] = 0.0
    f.ravel()[2] = np.inf
    f.ravel()[3] = -np.inf
    r = oracle.vertex_order(f)
    g = f.ravel().copy()
    g[g == 0] = 0.0
    expect = np.empty(g.size, dtype=np.int64)
    expect[np.argsort(g, kind="stable")] = np.arange(g.size)
    assert np.array_equal(r, expect)


@pytest.mark.parametrize("field", [sf.with_infinities(sf.noise((6, 5, 7), 40), 40),
                                   sf.with_infinities(sf.gaussians((8, 7, 6), 41, 3, 0.01), 41, 0.3, 0.1)])
def test_infinities_match_bruteforce(field):
    # +-inf are ordinary, ordered values (ties by index); the whole pipeline
    # on such a field equals the full-filtration reduction
    g = field.ravel()
    expect = np.empty(g.size, dtype=np.int64)
    expect[np.argsort(g, kind="stable")] = np.arange(g.size)
    assert np.array_equal(oracle.vertex_order(field), expect)
    _bf_equal(field)


def test_vertex_order_rejects_nan():
    f = sf.noise((3, 3, 3), 0)
    f[1, 1, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.vertex_order(f)
    with pytest.raises(ValueError):
        oracle.run(f)


def test_bruteforce_every_order_of_one_cube():
    """All 8! = 40320 vertex orders of the 2x2x2 grid (51 simplices)."""
    for perm in itertools.permutations(range(8)):
        f = np.array(perm, dtype=np.float32).reshape(2, 2, 2)
        res = _bf_equal(f)
        c = [len(x) for x in res.crit]
        assert c[0] - c[1] + c[2] - c[3] == 1


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 4, 4), (2, 3, 4), (5, 3, 2), (3, 5, 4)])
def test_bruteforce_small_random_orders(shape):
    rng = np.random.default_rng(sum(shape))
    n = int(np.prod(shape))
    for _ in range(40):
        _bf_equal(rng.permutation(n).astype(np.float32).reshape(shape))


def test_bruteforce_small_with_heavy_ties():
    rng = np.random.default_rng(11)
    for _ in range(40):
        _bf_equal(rng.integers(0, 3, size=(4, 4, 4)).astype(np.float32))


@pytest.mark.parametrize("seed", range(16))
def test_bruteforce_16cube_noise(seed):
    _bf_equal(sf.noise((16, 16, 16), seed))


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(16, 64))
def test_bruteforce_16cube_noise_more_seeds(seed):
    _bf_equal(sf.noise((16, 16, 16), seed))


def test_bruteforce_smooth_fields():
    _bf_equal(sf.gaussians((12, 14, 10), 5, k=6, noise_frac=0.01))
    _bf_equal(sf.gaussians((16, 16, 16), 6, k=8, noise_frac=0.0))


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(2))
def test_bruteforce_32cube(seed):
    _bf_equal(sf.noise((32, 32, 32), seed))


@pytest.mark.parametrize("field", [
    sf.noise((16, 16, 16), 7),
    sf.noise((5, 9, 7), 8),
    sf.gaussians((12, 12, 12), 9, k=5, noise_frac=0.02),
    sf.radial((9, 9, 9)),
])
def test_critical_cells_equal_lower_link_betti(field):
    res = oracle.run(field)
    betti = oracle.bf_lower_link_betti(res.shape, res.rank)
    counts = np.zeros_like(betti)
    for d in range(4):
        if len(res.crit[d]):
            mv = H.vertices(res.shape, d, res.crit[d])
            top = mv[np.arange(len(mv)), res.rank[mv].argmax(axis=1)]
            np.add.at(counts[:, d], top, 1)
    assert np.array_equal(counts, betti)


@pytest.mark.parametrize("field", [sf.noise((10, 9, 8), 2), sf.gaussians((10, 10, 10), 4, 4, 0.01)])
def test_gradient_is_a_valid_acyclic_matching(field):
    res = oracle.run(field)
    shape, rank = res.shape, res.rank
    for d in range(4):
        P = res.partner[d]
        ids = np.nonzero(P >= 0)[0]
        mates = P[ids]
        md, mid = mates & 3, mates >> 2
        assert np.all((md == d - 1) | (md == d + 1))
        # symmetric
        for dd in (d - 1, d + 1):
            sel = md == dd
            if sel.any():
                assert np.array_equal(res.partner[dd][mid[sel]], ids[sel] * 4 + d)
        # facet relation and same highest vertex (one lower star)
        up = md == d + 1
        if up.any():
            fs = H.facets(shape, d + 1, mid[up])
            assert np.all((fs == ids[up][:, None]).sum(axis=1) == 1)
            a = rank[H.vertices(shape, d, ids[up])].max(axis=1)
            b = rank[H.vertices(shape, d + 1, mid[up])].max(axis=1)
            assert np.array_equal(a, b)
    # acyclic v-paths for each level d -> d+1 (Kahn's algorithm on the
    # graph tail -> other facets of its head)
    for d in range(3):
        P = res.partner[d]
        tails = np.nonzero((P >= 0) & ((P & 3) == d + 1))[0]
        heads = P[tails] >> 2
        fs = H.facets(shape, d + 1, heads)
        succ = {}
        for t, row in zip(tails.tolist(), fs.tolist()):
            succ[t] = [x for x in row if x != t]
        indeg = {}
        for t, nxt in succ.items():
            for x in nxt:
                if x in succ:
                    indeg[x] = indeg.get(x, 0) + 1
        stack = [t for t in succ if indeg.get(t, 0) == 0]
        seen = 0
        while stack:
            t = stack.pop()
            seen += 1
            for x in succ[t]:
                if x in succ:
                    indeg[x] -= 1
                    if indeg[x] == 0:
                        stack.append(x)
        assert seen == len(succ), f"closed v-path among {d}-simplices"


@pytest.mark.parametrize("coeffs", [(1.0, 1.7320508, 2.2360679), (0.3, 0.11, 0.7)])
def test_elevation_has_one_essential_class_only(coeffs):
    """A linear ramp has a single critical cell, the lowest corner: D0 holds
    one infinite class and D1 = D2 = empty (the 'Elevation' case)."""
    f = sf.elevation((7, 6, 5), coeffs)
    res = oracle.run(f)
    assert [len(c) for c in res.crit] == [1, 0, 0, 0]
    assert res.crit[0].tolist() == [0]
    assert res.pairs[0].tolist() == [[0, -1]]
    assert res.pairs[1].size == 0 and res.pairs[2].size == 0
    g = -f
    res = oracle.run(g)
    assert res.crit[0].tolist() == [f.size - 1]
    assert [len(c) for c in res.crit] == [1, 0, 0, 0]


def test_radial_field_significant_pairs():
    """f = -|p - c|^2 on the cube: 8 corner minima merge through the 12 edge
    saddles (7 deaths, 5 loops), the 6 face saddles close 5 loops and form
    one void that the central maximum fills. Pairs of large persistence
    therefore number 7 / 5 / 1 in D0 / D1 / D2."""
    f = sf.radial((17, 17, 17))
    res = oracle.run(f)
    fv = f.ravel()
    span = float(fv.max() - fv.min())
    big = []
    for d in range(3):
        p = res.pairs[d]
        fin = p[p[:, 1] >= 0]
        b = fv[oracle.simplex_vertices(res.shape, d, fin[:, 0])].max(axis=1)
        e = fv[oracle.simplex_vertices(res.shape, d + 1, fin[:, 1])].max(axis=1)
        big.append(int(((e - b) > 0.05 * span).sum()))
    assert big == [7, 5, 1]
    _bf_equal(f)


@pytest.mark.parametrize("field", [sf.noise((16, 16, 16), 21), sf.gaussians((20, 18, 16), 3, 10, 0.01),
                                   sf.noise((2, 2, 9), 4)])
def test_invariants(field):
    res = oracle.run(field)
    c = [len(x) for x in res.crit]
    assert c[0] - c[1] + c[2] - c[3] == 1
    d0, d1, d2 = res.pairs
    assert int((d0[:, 1] < 0).sum()) == 1 and (d1[:, 1] >= 0).all() and (d2[:, 1] >= 0).all()
    ess = d0[d0[:, 1] < 0, 0]
    assert res.rank[ess[0]] == 0  # the global minimum
    assert len(d0) - 1 == c[0] - 1
    assert len(d2) == c[3]
    assert len(d1) == c[1] - (c[0] - 1) == c[2] - c[3]
    # every pair is born before it dies in the lexicographic order
    for d in range(3):
        fin = res.pairs[d][res.pairs[d][:, 1] >= 0]
        kb = np.sort(res.rank[oracle.simplex_vertices(res.shape, d, fin[:, 0])], axis=1)[:, ::-1]
        kd = np.sort(res.rank[oracle.simplex_vertices(res.shape, d + 1, fin[:, 1])], axis=1)[:, ::-1]
        for x, y in zip(kb.tolist(), kd.tolist()):
            assert x < y[: len(x)] or (x == y[: len(x)])


def test_noise_extrema_statistics():
    """i.i.d. continuous noise: a vertex is a minimum with probability
    1/(deg+1); an interior vertex is a maximum (a critical tetrahedron) with
    probability 1/15. Means over seeds must sit within 4 sigma."""
    shape = (16, 16, 16)
    deg = np.zeros(shape, dtype=np.int64)
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        if (dz, dy, dx) == (0, 0, 0):
            continue
        if not ((dx, dy, dz) in [(a * s, b * s, c * s) for s in (1, -1) for a, b, c in
                                 itertools.product((0, 1), repeat=3) if a + b + c]):
            continue
        ok = np.ones(shape, dtype=bool)
        for ax, dd in zip((0, 1, 2), (dz, dy, dx)):
            idx = np.arange(shape[ax])
            m = (idx + dd >= 0) & (idx + dd < shape[ax])
            sl = [None, None, None]
            sl[ax] = slice(None)
            ok &= m[tuple(sl)]
        deg += ok
    e_min = float((1.0 / (deg + 1)).sum())
    e_max = 14 ** 3 / 15.0
    mins, maxs = [], []
    for seed in range(24):
        res = oracle.run(sf.noise(shape, 100 + seed))
        mins.append(len(res.crit[0]))
        maxs.append(len(res.crit[3]))
    assert abs(e_min - 312.63) < 0.01
    assert abs(np.mean(mins) - e_min) < 4 * np.sqrt(e_min / len(mins))
    assert abs(np.mean(maxs) - e_max) < 4 * np.sqrt(e_max / len(maxs))


def test_golden_simplex_counts():
    """tests/golden/simplex_counts.json (closed forms) against the brute-force
    enumeration of all faces of all Kuhn tetrahedra."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "simplex_counts.json")
    gold = json.load(open(path))
    for key, val in gold.items():
        nx, ny, nz = map(int, key.split("x"))
        if nx * ny * nz <= 4096:
            assert list(oracle.bf_counts((nz, ny, nx))) == val, key
    assert gold["512x512x512"] == [134217728, 936381439, 1602760698, 800596986]


@pytest.mark.parametrize("field", [sf.noise((16, 16, 16), 31), sf.gaussians((20, 18, 16), 2, 6, 0.01),
                                   sf.noise((3, 7, 5), 1)])
def test_kruskal_d0_matches_oracle(field):
    """The Kruskal checker used at full size agrees with the oracle's D0 (and
    so, by the brute-force pins, with boundary-matrix reduction)."""
    res = oracle.run(field)
    fin, _ = oracle.order_space(res)
    d0 = sorted((b, d) for (dim, b, d) in fin if dim == 0)
    assert d0 == [tuple(x) for x in oracle.bf_d0_kruskal(res.shape, res.rank).tolist()]


@pytest.mark.parametrize("field", [sf.noise((16, 16, 16), 32), sf.gaussians((12, 14, 10), 3, 5, 0.01),
                                   sf.radial((17, 17, 17)), sf.noise((2, 2, 9), 4), sf.noise((3, 17, 2), 5),
                                   sf.with_infinities(sf.noise((6, 7, 5), 6), 6),
                                   np.random.default_rng(7).integers(0, 3, size=(7, 6, 8)).astype(np.float32)])
def test_dual_d2_matches_bruteforce_and_oracle(field):
    """The dual union-find checker used at full size (every triangle and
    tetrahedron, outside node, Sec. 5.2) gives the D2 of the full boundary
    reduction, and the oracle's D2 equals both."""
    res = oracle.run(field)
    bp, _ = oracle.bf_diagram(res.shape, res.rank)
    exp = sorted((int(b), int(d)) for dd, b, d in bp.tolist() if dd == 2)
    got = [tuple(x) for x in oracle.bf_d2_dual(res.shape, res.rank).tolist()]
    assert got == exp
    fin, _ = oracle.order_space(res)
    assert sorted((b, d) for (dim, b, d) in fin if dim == 2) == exp


def test_dual_d2_every_order_of_one_cube_and_random_orders():
    """Every vertex order of one cube (its D2 is a single void at most) and
    random orders of small grids: dual union-find = full reduction."""
    for perm in itertools.permutations(range(8)):
        r = np.array(perm, dtype=np.uint32)
        bp, _ = oracle.bf_diagram((2, 2, 2), r)
        exp = sorted((int(b), int(d)) for dd, b, d in bp.tolist() if dd == 2)
        assert [tuple(x) for x in oracle.bf_d2_dual((2, 2, 2), r).tolist()] == exp, perm
    rng = np.random.default_rng(8)
    for shape in [(3, 3, 3), (4, 3, 5), (2, 4, 3)]:
        for _ in range(40):
            r = rng.permutation(int(np.prod(shape))).astype(np.uint32)
            bp, _ = oracle.bf_diagram(shape, r)
            exp = sorted((int(b), int(d)) for dd, b, d in bp.tolist() if dd == 2)
            assert [tuple(x) for x in oracle.bf_d2_dual(shape, r).tolist()] == exp, shape


@pytest.mark.parametrize("field", [sf.noise((16, 16, 16), 0), sf.noise((24, 24, 24), 3),
                                   sf.gaussians((20, 22, 18), 7, k=8, noise_frac=0.01),
                                   np.random.default_rng(6).integers(0, 4, size=(9, 8, 7)).astype(np.float32)])
def test_sandwich_does_not_change_d1(field):
    """Sec. 3: restricting PairCriticalSimplices to the 2-saddles D2 left
    unpaired gives the D1 of running it on every critical triangle (where the
    triangles D2 pairs reduce to an empty boundary)."""
    a = oracle.run(field)
    b = oracle.run(field, sandwich=False)
    for d in range(3):
        assert np.array_equal(a.pairs[d], b.pairs[d])
    st = oracle.bf_check_cycles(a.shape, a.rank, b.pairs[1][b.pairs[1][:, 1] >= 0], b.gen1_off, b.gen1_edges)
    assert (st == 0).all()


@pytest.mark.parametrize("field", [sf.noise((16, 16, 16), 0), sf.gaussians((20, 22, 18), 7, k=8, noise_frac=0.01),
                                   np.random.default_rng(6).integers(0, 4, size=(9, 8, 7)).astype(np.float32)])
def test_caching_does_not_change_d1(field):
    """Sec. 4.1(b): adding an earlier 2-saddle's own boundary and reducing it
    again gives the pairs of adding its cached reduced boundary, with or
    without the sandwich; it only takes more additions."""
    a = oracle.run(field)
    for sandwich in (True, False):
        b = oracle.run(field, sandwich=sandwich, cache=False)
        for d in range(3):
            assert np.array_equal(a.pairs[d], b.pairs[d]), (sandwich, d)
        assert b.d1_adds >= oracle.run(field, sandwich=sandwich).d1_adds


def test_sandwich_ablation_needs_the_virtual_maximum():
    """Without the outside node (App. A) D2 from the dual union-find is not
    the plain reduction's, so D1 over every critical triangle is another
    computation: the oracle refuses the combination."""
    with pytest.raises(ValueError):
        oracle.run(sf.noise((6, 6, 6), 0), sandwich=False, virtual_max=False)
