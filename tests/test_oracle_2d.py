"""Pins of the oracle on 2D grids (nz = 1, the plane z = 0 of the same
triangulation), CPU only.

On a 2D grid the method takes D0 from the unstable sets of the 1-saddles and
D1 from their stable sets with the dual union-find (Sec. 3, 5); there is no
sandwich. The brute-force checker builds the complex from the grid's
triangles and reduces the whole lexicographic filtration: the diagrams must
agree in vertex-order space, for every vertex order of a small grid and for
random, tied, thin and smooth fields.
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


def _counts2d(ny, nx):
    V = nx * ny
    E = (nx - 1) * ny + nx * (ny - 1) + (nx - 1) * (ny - 1)
    T = 2 * (nx - 1) * (ny - 1)
    return V, E, T


@pytest.mark.parametrize("shape", [(1, 2, 2), (1, 3, 7), (1, 16, 9)])
def test_counts_2d_closed_form(shape):
    c = oracle.bf_counts(shape)
    V, E, T = _counts2d(shape[1], shape[2])
    assert list(c) == [V, E, T, 0]
    assert V - E + T == 1


def test_every_order_of_a_2x3_grid():
    for perm in itertools.permutations(range(6)):
        res = _bf_equal(np.array(perm, dtype=np.float32).reshape(1, 2, 3))
        c = [len(x) for x in res.crit]
        assert c[3] == 0 and c[0] - c[1] + c[2] == 1


@pytest.mark.parametrize("shape", [(1, 3, 3), (1, 4, 5), (1, 2, 9), (1, 6, 6)])
def test_random_orders_2d(shape):
    rng = np.random.default_rng(sum(shape))
    n = int(np.prod(shape))
    for _ in range(60):
        _bf_equal(rng.permutation(n).astype(np.float32).reshape(shape))


@pytest.mark.parametrize("field", ["noise", "smooth", "ties", "thin"])
def test_fields_2d(field):
    f = {
        "noise": lambda: sf.noise((1, 33, 17), 4),
        "smooth": lambda: sf.gaussians((1, 48, 40), 3, k=8, noise_frac=0.01),
        "ties": lambda: np.random.default_rng(6).integers(0, 4, size=(1, 12, 11)).astype(np.float32),
        "thin": lambda: sf.noise((1, 2, 40), 5),
    }[field]()
    res = _bf_equal(f)
    c = [len(x) for x in res.crit]
    d0, d1, d2 = res.pairs
    # Euler characteristic of the square; one infinite class, at the global
    # minimum; every maximum dies in D1; no D2
    assert c[3] == 0 and c[0] - c[1] + c[2] == 1
    assert len(d0) == c[0] and (d0[:-1, 1] >= 0).all() and d0[-1, 1] == -1
    assert res.rank[d0[-1, 0]] == 0
    assert len(d1) == c[2] == c[1] - c[0] + 1 and (d1[:, 1] >= 0).all()
    assert len(d2) == 0


def test_2d_gradient_pairs_are_lower_star_facet_pairs():
    """Definition of the discrete gradient on a 2D grid: every pair is a
    facet/cofacet pair inside one lower star (same highest vertex), the
    matching is symmetric, and there are no tetrahedra."""
    f = sf.noise((1, 10, 12), 7)
    res = oracle.run(f)
    shape = res.shape
    for dim in (0, 1):
        P = res.partner[dim]
        ids = np.nonzero(P >= 0)[0]
        for i in ids:
            p = int(P[i])
            pd, pid = p & 3, p >> 2
            assert pd in (dim - 1, dim + 1)
            back = res.partner[pd][pid]
            assert back == i * 4 + dim
            a = oracle.simplex_vertices(shape, dim, np.array([i]))[0]
            b = oracle.simplex_vertices(shape, pd, np.array([pid]))[0]
            small, big = (a, b) if pd > dim else (b, a)
            assert set(small) <= set(big)
            # same lower star: the highest vertex is shared
            assert max(res.rank[small]) == max(res.rank[big])
    # no tetrahedra, and every existing triangle lies in the plane
    assert (res.partner[3] == -2).all()


@pytest.mark.parametrize("field", ["noise", "smooth", "ties", "thin"])
def test_2d_critical_cells_equal_lower_link_betti(field):
    """The expansion-based gradient puts exactly b~_{k-1}(lower link) critical
    k-cells in each lower star (Sec. 1.1, 2.6); on a 2D grid the link of a
    vertex is the cycle of its (up to) six neighbours."""
    f = {
        "noise": lambda: sf.noise((1, 21, 19), 12),
        "smooth": lambda: sf.gaussians((1, 40, 36), 13, k=6, noise_frac=0.01),
        "ties": lambda: np.random.default_rng(14).integers(0, 3, size=(1, 15, 16)).astype(np.float32),
        "thin": lambda: sf.noise((1, 2, 30), 15),
    }[field]()
    res = oracle.run(f)
    betti = oracle.bf_lower_link_betti(res.shape, res.rank)
    counts = np.zeros_like(betti)
    for d in range(3):
        if len(res.crit[d]):
            mv = H.vertices(res.shape, d, res.crit[d])
            top = mv[np.arange(len(mv)), res.rank[mv].argmax(axis=1)]
            np.add.at(counts[:, d], top, 1)
    assert np.array_equal(counts, betti)
