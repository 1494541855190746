"""A model of the lock-free PairCriticalSimplices rule (Sec. 7.2), on the CPU.

The GPU reduces all the 2-saddles D2 left unpaired at once: a column whose
highest edge tau is regular adds the boundary of tau's gradient triangle;
if tau is critical it claims tau when nobody owns it, adds the boundary an
earlier owner published (looking again if that owner moved on), or evicts a
later owner and carries that column on. This test replays the rule step by
step in Python with random interleavings of many lanes and checks the pairs
against the oracle's sequential D1, and each published cycle against the
definition of a generator. It shares no code with the kernels.
"""
import numpy as np
import pytest

import oracle
import synthfields as sf
from tests import helpers as H


def _model(res, lanes, rng, evict=True):
    shape = res.shape
    rank = res.rank.astype(np.int64)
    c2 = res.crit[2]
    paired2 = set(int(t) for t, m in res.pairs[2] if m >= 0)
    cols = [int(t) for t in c2 if int(t) not in paired2]  # ascending: column order
    partner1 = res.partner[1]
    ev = H.vertices(shape, 1, np.arange(len(partner1)))

    def ekey(e):
        a, b = rank[ev[e, 0]], rank[ev[e, 1]]
        return (max(a, b), min(a, b))

    def bd(t):
        return set(int(e) for e in H.facets(shape, 2, np.array([t]))[0])

    owner, published = {}, {}
    state = [None] * lanes  # [column, boundary set]
    nxt, steps = 0, 0
    while True:
        for i in range(lanes):
            if state[i] is None and nxt < len(cols):
                state[i] = [nxt, bd(cols[nxt])]
                nxt += 1
        active = [i for i in range(lanes) if state[i] is not None]
        if not active:
            break
        i = active[rng.integers(len(active))]
        c, B = state[i]
        steps += 1
        assert steps < 10 ** 7 and B, "boundary vanished"
        tau = max(B, key=ekey)
        p = int(partner1[tau])
        if p >= 0:  # regular: add the boundary of its gradient triangle
            assert p & 3 == 2
            B ^= bd(p >> 2)
            continue
        o = owner.get(tau)
        if o is None:
            published[c] = frozenset(B)
            owner[tau] = c
            state[i] = None
        elif o < c or not evict:
            P = published[o]
            if max(P, key=ekey) != tau:  # the owner moved on; look again
                continue
            B ^= P
        else:  # o > c: take tau, carry the evicted column on
            published[c] = frozenset(B)
            owner[tau] = c
            state[i] = [o, set(published[o])]
    return {(tau, cols[c]) for tau, c in owner.items()}, {cols[c]: z for c, z in published.items()}


@pytest.mark.parametrize("field,lanes", [(sf.noise((8, 8, 8), 4), 1), (sf.noise((8, 8, 8), 4), 16),
                                         (sf.noise((9, 10, 8), 5), 64),
                                         (sf.gaussians((12, 12, 12), 6, k=5, noise_frac=0.03), 32)])
def test_interleaved_pair_critical_simplices_gives_the_sequential_pairs(field, lanes):
    res = oracle.run(field)
    d1 = res.pairs[1]
    expect = {(int(e), int(t)) for e, t in d1 if t >= 0}
    for seed in range(3):
        got, cycles = _model(res, lanes, np.random.default_rng(seed))
        assert got == expect, (lanes, seed)
        # the cycle each 2-saddle published when it took its final pivot
        fin = np.array(sorted(expect), dtype=np.int64).reshape(-1, 2)
        zs = [np.array(sorted(cycles[int(t)]), dtype=np.int64) for _, t in fin]
        off = np.zeros(len(zs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(z) for z in zs])
        st = oracle.bf_check_cycles(res.shape, res.rank, fin, off, np.concatenate(zs))
        assert (st == 0).all()


def test_adding_a_later_owner_instead_of_evicting_it_goes_wrong():
    """Planted mistake: a column that adds the boundary of a later owner (a
    right-to-left operation) instead of taking the pivot gives other pairs."""
    res = oracle.run(sf.noise((9, 10, 8), 5))
    expect = {(int(e), int(t)) for e, t in res.pairs[1] if t >= 0}
    wrong = 0
    for seed in range(3):
        try:
            got, _ = _model(res, 64, np.random.default_rng(seed), evict=False)
            wrong += got != expect
        except AssertionError:  # a boundary vanished or no progress
            wrong += 1
    assert wrong == 3
