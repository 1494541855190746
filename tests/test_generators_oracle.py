"""Persistent 1-cycle generators of the oracle against their definition (CPU).

For a D1 pair (tau, sigma) the method keeps the boundary it cached when sigma
was paired: a 1-cycle homologous to the boundary of sigma and born at tau
(Sec. 8). The brute-force checker rebuilds the whole lexicographic
filtration from the tetrahedra and checks each cycle: even degree at every
vertex, highest edge tau, and cycle + boundary(sigma) a sum of boundaries of
triangles that come before sigma (Z2 elimination). Planted mistakes show that
each of the three conditions is really tested.
"""
import numpy as np
import pytest

import oracle
import synthfields as sf

FIELDS = {
    "noise567": lambda: sf.noise((5, 6, 7), 0),
    "noise8": lambda: sf.noise((8, 8, 8), 3),
    "noise_thin": lambda: sf.noise((2, 3, 11), 4),
    "smooth12": lambda: sf.gaussians((12, 11, 10), 5, k=6, noise_frac=0.02),
    "ties": lambda: np.random.default_rng(6).integers(0, 4, size=(9, 8, 7)).astype(np.float32),
    "noise16": lambda: sf.noise((16, 16, 16), 6),
}


def _finite(res):
    p1 = res.pairs[1]
    return p1[p1[:, 1] >= 0]


@pytest.mark.parametrize("name", sorted(FIELDS))
def test_oracle_generators_valid(name):
    res = oracle.run(FIELDS[name]())
    fin = _finite(res)
    assert len(res.gen1_off) == len(fin) + 1
    assert res.gen1_off[-1] == len(res.gen1_edges)
    st = oracle.bf_check_cycles(res.shape, res.rank, fin, res.gen1_off, res.gen1_edges)
    assert (st == 0).all(), np.bincount(st)
    # the birth edge is in its own cycle; edge ids ascending within a cycle
    for i, (tau, _) in enumerate(fin):
        z = res.gen1_edges[res.gen1_off[i]:res.gen1_off[i + 1]]
        assert tau in z
        assert (np.diff(z) > 0).all()


def _gens(res):
    return [res.gen1_edges[res.gen1_off[i]:res.gen1_off[i + 1]].copy() for i in range(len(res.gen1_off) - 1)]


def _pack(gens):
    off = np.zeros(len(gens) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(g) for g in gens])
    return off, (np.concatenate(gens) if gens else np.zeros(0, dtype=np.int64))


def _edge_key(res, e):
    vs = oracle.simplex_vertices(res.shape, 1, np.array([e]))[0]
    return tuple(sorted((int(res.rank[v]) for v in vs), reverse=True))


def _tri_key(res, t):
    vs = oracle.simplex_vertices(res.shape, 2, np.array([t]))[0]
    return tuple(sorted((int(res.rank[v]) for v in vs), reverse=True))


def test_checker_catches_planted_mistakes():
    res = oracle.run(sf.noise((8, 8, 8), 3))
    fin = _finite(res)
    gens = _gens(res)
    n = len(fin)
    assert n > 4
    # 1. an edge dropped from a cycle of more than three edges: not a cycle
    i = next(k for k in range(n) if len(gens[k]) > 3)
    bad = list(gens)
    z = gens[i]
    bad[i] = z[z != z[0]] if z[0] != fin[i, 0] else z[z != z[1]]
    st = oracle.bf_check_cycles(res.shape, res.rank, fin, *_pack(bad))
    assert st[i] == 1 and (np.delete(st, i) == 0).all()
    # 2. two cycles swapped: a valid cycle, but not born at tau
    bad = list(gens)
    bad[0], bad[1] = gens[1], gens[0]
    st = oracle.bf_check_cycles(res.shape, res.rank, fin, *_pack(bad))
    assert st[0] == 3 and st[1] == 3 and (st[2:] == 0).all()
    # 3. a nested pair (tau_j < tau_i, sigma_j > sigma_i): z_i + z_j is a cycle
    # born at tau_i, but z_j is still alive at sigma_i, so it is not
    # homologous to boundary(sigma_i) before sigma_i
    ek = [_edge_key(res, t) for t in fin[:, 0]]
    tk = [_tri_key(res, s) for s in fin[:, 1]]
    nested = [(a, b) for a in range(n) for b in range(n) if ek[b] < ek[a] and tk[b] > tk[a]]
    assert nested, "no nested D1 pairs in this field"
    a, b = nested[0]
    bad = list(gens)
    bad[a] = np.setxor1d(gens[a], gens[b])
    st = oracle.bf_check_cycles(res.shape, res.rank, fin, *_pack(bad))
    assert st[a] == 4 and (np.delete(st, a) == 0).all()
    # 4. adding a cycle that is already dead by sigma_i is harmless: a pair
    # born and killed earlier (tau_j < tau_i, sigma_j < sigma_i)
    earlier = [(a, b) for a in range(n) for b in range(n) if ek[b] < ek[a] and tk[b] < tk[a]]
    assert earlier
    a, b = earlier[0]
    good = list(gens)
    good[a] = np.setxor1d(gens[a], gens[b])
    st = oracle.bf_check_cycles(res.shape, res.rank, fin, *_pack(good))
    assert (st == 0).all()


def test_generators_every_order_of_one_cube():
    """Every vertex order of one cube: each D1 pair's cycle passes the check."""
    import itertools
    n_pairs = 0
    for perm in itertools.permutations(range(8)):
        res = oracle.run(np.array(perm, dtype=np.float32).reshape(2, 2, 2))
        fin = _finite(res)
        if len(fin):
            st = oracle.bf_check_cycles(res.shape, res.rank, fin, res.gen1_off, res.gen1_edges)
            assert (st == 0).all(), (perm, st)
            n_pairs += len(fin)
    assert n_pairs > 0


@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 4, 4), (2, 3, 5)])
def test_generators_random_orders(shape):
    rng = np.random.default_rng(100 + sum(shape))
    n = int(np.prod(shape))
    for _ in range(60):
        res = oracle.run(rng.permutation(n).astype(np.float32).reshape(shape))
        fin = _finite(res)
        st = oracle.bf_check_cycles(res.shape, res.rank, fin, res.gen1_off, res.gen1_edges)
        assert (st == 0).all()
