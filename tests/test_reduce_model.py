"""A model of the lock-free two-entry reduction with path halving (CPU).

The GPU reduces the D0 (and D2) arcs as two-entry columns, all at once:
columns claim their pivot, add the published boundary of an earlier owner,
evict a later owner and carry its column on, and follow path-halving
shortcuts jump[p] = (r, M), each usable only by a column after M. This test
replays that rule step by step in Python, with a random interleaving of many
lanes, and checks that the pairs equal the oracle's union-find. It shares no
code with the kernel; it checks the argument (every step adds a sum of
columns to the left) under interleavings the GPU tests only sample.
"""
import numpy as np
import pytest

import oracle
import synthfields as sf

EMPTY = -1


def _reduce_interleaved(na, nb, lanes, rng, bound=True, drop=None):
    m = len(na)
    owner = {}
    bnd = [None] * m
    jump = {}
    nxt = 0
    state = [None] * lanes  # per lane: [c, p, q, pp, pm] or None
    steps = 0
    while True:
        active = [i for i in range(lanes) if state[i] is not None]
        if nxt < m:
            idle = [i for i in range(lanes) if state[i] is None]
            for i in idle:
                while nxt < m and drop is not None and drop(nxt):
                    nxt += 1  # a column left out: unpaired, the lane takes the next one
                if nxt < m:
                    p, q = max(na[nxt], nb[nxt]), min(na[nxt], nb[nxt])
                    state[i] = [nxt, p, q, EMPTY, 0]
                    nxt += 1
            active = [i for i in range(lanes) if state[i] is not None]
        if not active:
            break
        i = active[rng.integers(len(active))]
        c, p, q, pp, pm = state[i]
        steps += 1
        assert steps < 50 * m * m + 1000
        if p == q:  # reduced to zero
            state[i] = None
            continue
        o = owner.get(p, EMPTY)
        if o == EMPTY:
            bnd[c] = (p, q)
            owner[p] = c  # the compare-and-swap succeeds: nothing ran in between
            state[i] = None
            continue
        if o < c:
            sc = jump.get(p)
            if sc is not None and (sc[1] < c or not bound):
                r, M = sc
            else:
                bp, bq = bnd[o]
                if bp != p:  # the owner moved on; look again
                    continue
                r, M = bq, o
            if pp != EMPTY:
                jump[pp] = (r, max(pm, M))
            if q > r:
                state[i] = [c, q, r, EMPTY, 0]
            else:
                state[i] = [c, r, q, p, M]
            continue
        # o > c: c takes the pivot, the lane carries the evicted column on
        bnd[c] = (p, q)
        owner[p] = c
        op, oq = bnd[o]
        state[i] = [o, op, oq, EMPTY, 0]
    return owner


@pytest.mark.parametrize("field,lanes", [(sf.noise((10, 10, 10), 1), 1), (sf.noise((10, 10, 10), 1), 7),
                                         (sf.noise((12, 11, 10), 2), 64),
                                         (sf.gaussians((14, 14, 14), 3, k=5, noise_frac=0.02), 32)])
def test_interleaved_reduction_with_path_halving_gives_the_union_find_pairs(field, lanes):
    res = oracle.run(field)
    rank = res.rank.astype(np.int64)
    na = [int(rank[a]) for a in res.arcs0[:, 0]]
    nb = [int(rank[b]) for b in res.arcs0[:, 1]]
    edges = res.arcs0[:, 2]
    expect = {(int(rank[b]), int(e)) for b, e in res.pairs[0] if e >= 0}
    for seed in range(3):
        owner = _reduce_interleaved(na, nb, lanes, np.random.default_rng(seed))
        got = {(p, int(edges[c])) for p, c in owner.items()}
        assert got == expect, (lanes, seed)


def test_the_column_bound_of_the_shortcuts_is_needed():
    """Planted mistake: shortcuts used by columns before their bound M add
    sums that include columns to the right, and the pairs go wrong."""
    res = oracle.run(sf.noise((12, 11, 10), 2))
    rank = res.rank.astype(np.int64)
    na = [int(rank[a]) for a in res.arcs0[:, 0]]
    nb = [int(rank[b]) for b in res.arcs0[:, 1]]
    edges = res.arcs0[:, 2]
    expect = {(int(rank[b]), int(e)) for b, e in res.pairs[0] if e >= 0}
    wrong = 0
    for seed in range(10):
        try:
            owner = _reduce_interleaved(na, nb, 64, np.random.default_rng(seed), bound=False)
            wrong += {(p, int(edges[c])) for p, c in owner.items()} != expect
        except AssertionError:  # no progress
            wrong += 1
    assert wrong > 0


@pytest.mark.parametrize("virtual_max", [True, False])
@pytest.mark.parametrize("field,lanes", [(sf.noise((10, 10, 10), 1), 16), (sf.noise((12, 11, 10), 2), 64),
                                         (sf.with_infinities(sf.noise((7, 8, 9), 9), 9), 32)])
def test_dual_reduction_both_boundary_modes(field, lanes, virtual_max):
    """The D2 arcs reduced the same way, the outside as node 0 (the oldest):
    with the virtual maximum every column takes part; without it a column
    with an end outside is left out (the lane takes the next column at once).
    The pairs equal the oracle's dual union-find in the same mode."""
    res = oracle.run(field, virtual_max=virtual_max)
    tets = res.crit[3]
    age = {int(t): len(tets) - i for i, t in enumerate(tets)}  # 1 = the highest maximum
    na = [0 if a < 0 else age[int(a)] for a in res.arcs2[:, 0]]
    nb = [0 if b < 0 else age[int(b)] for b in res.arcs2[:, 1]]
    tri = res.arcs2[:, 2]
    expect = {(int(t), int(T)) for t, T in res.pairs[2] if T >= 0}
    drop = None if virtual_max else (lambda c: na[c] == 0 or nb[c] == 0)
    for seed in range(3):
        owner = _reduce_interleaved(na, nb, lanes, np.random.default_rng(seed), drop=drop)
        got = {(int(tri[c]), int(tets[len(tets) - p])) for p, c in owner.items() if p != 0}
        assert got == expect, (lanes, seed, virtual_max)
