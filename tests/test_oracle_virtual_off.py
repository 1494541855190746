"""The oracle without the virtual maximum on the domain boundary (the
optional adjustment of Sec. 5.2 switched off; App. A, "Boundary
perturbations"). The mode is not a plain definition (it is the paper's
algorithm run as is with the outside removed from the dual union-find), so it
is pinned by what the reading fixes:

* D0 does not depend on the boundary mode;
* every critical simplex is accounted for exactly once (a birth, a death or
  an infinite class), and the global maximum is never killed;
* every finite D2 pair comes from a saddle whose two sides reach maxima (no
  arc to the outside), so they are a subset of the dual union-find's work;
* hand-built fields where the outcome is known: a radial field (3D: the
  highest face-centre 2-saddle, which kills the maximum with the virtual
  maximum on, becomes an infinite D2 class and D1 is unchanged; 2D: the
  highest saddle becomes an infinite D1 class and the maximum an infinite D2
  class), two bumps in the cube (the internal saddle still kills the lower
  bump; the boundary saddle that killed the global maximum becomes an
  infinite class -- the situation of App. A), a linear ramp (no change).
"""
import numpy as np
import pytest

import oracle
import synthfields as sf


def _bumps(n, a1=1.0, a2=0.7, sep=0.18, s=0.09):
    z, y, x = np.meshgrid(*[np.arange(n) / (n - 1)] * 3, indexing="ij")
    g = a1 * np.exp(-((x - 0.5 + sep) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / (2 * s * s))
    g += a2 * np.exp(-((x - 0.5 - sep) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / (2 * s * s))
    g += 1e-3 * (x + 1.7 * y + 2.3 * z)  # generic: no ties
    return g.astype(np.float32)


FIELDS = {
    "noise": lambda: sf.noise((12, 11, 10), 1),
    "noise16": lambda: sf.noise((16, 16, 16), 3),
    "smooth": lambda: sf.gaussians((20, 18, 16), 2, 6, 0.01),
    "ties": lambda: np.random.default_rng(6).integers(0, 4, size=(9, 8, 7)).astype(np.float32),
    "thin": lambda: sf.noise((2, 5, 9), 4),
    "bumps": lambda: _bumps(20),
    "radial": lambda: sf.radial((17, 17, 17)),
    "noise2d": lambda: sf.noise((1, 40, 37), 5),
    "smooth2d": lambda: sf.gaussians((1, 64, 48), 6, 8, 0.01),
    "radial2d": lambda: sf.radial((1, 17, 17)),
}


@pytest.mark.parametrize("name", sorted(FIELDS))
def test_d0_and_accounting(name):
    f = FIELDS[name]()
    on, off = oracle.run(f), oracle.run(f, virtual_max=False)
    assert np.array_equal(on.pairs[0], off.pairs[0])
    c = [len(x) for x in off.crit]
    fin = [int((p[:, 1] >= 0).sum()) for p in off.pairs]
    ess = [int((p[:, 1] < 0).sum()) for p in off.pairs]
    flat = f.shape[0] == 1
    assert ess[0] == 1 and len(off.pairs[0]) == c[0]
    # edges: D0 deaths + D1 births (finite or not)
    assert c[1] == fin[0] + len(off.pairs[1])
    if flat:
        # triangles: dual D1 deaths + maxima never killed; the global maximum is one of them
        assert c[2] == fin[1] + ess[2] and ess[2] >= 1
        top = off.crit[2][-1]
        assert (off.pairs[2][:, 0] == top).any()
    else:
        # triangles: D1 deaths + D2 births (finite or not); tetrahedra: D2 deaths + never killed
        assert c[2] == fin[1] + len(off.pairs[2])
        if c[3]:  # (a grid two vertices thick has its maxima on the boundary only: no critical tetrahedron)
            assert c[3] >= fin[2] + 1
            assert off.crit[3][-1] not in set(off.pairs[2][:, 1].tolist())  # the global maximum survives
    # a finite pair of the dual union-find comes from a saddle with two inner sides
    dual = 1 if flat else 2
    arcs = {int(s): (a, b) for a, b, s in off.arcs2}
    for s, _ in off.pairs[dual][off.pairs[dual][:, 1] >= 0] if not flat else off.pairs[1][off.pairs[1][:, 1] >= 0]:
        a, b = arcs[int(s)]
        assert a >= 0 and b >= 0, (name, s)


def test_radial_3d():
    f = sf.radial((17, 17, 17))
    on, off = oracle.run(f), oracle.run(f, virtual_max=False)
    assert np.array_equal(on.pairs[1], off.pairs[1])
    assert len(on.pairs[2]) == 1 and on.pairs[2][0, 1] >= 0
    assert off.pairs[2].tolist() == [[int(on.pairs[2][0, 0]), -1]]


def test_radial_2d():
    f = sf.radial((1, 17, 17))
    on, off = oracle.run(f), oracle.run(f, virtual_max=False)
    fin_on = on.pairs[1][on.pairs[1][:, 1] >= 0]
    assert len(fin_on) == 1 and len(on.pairs[2]) == 0
    assert off.pairs[1].tolist() == [[int(fin_on[0, 0]), -1]]
    assert off.pairs[2].tolist() == [[int(fin_on[0, 1]), -1]]


def test_two_bumps_global_maximum():
    f = _bumps(24)
    on, off = oracle.run(f), oracle.run(f, virtual_max=False)
    assert np.array_equal(on.pairs[1], off.pairs[1])
    top = int(on.crit[3][-1])
    glob = [p for p in on.pairs[2].tolist() if p[1] == top]
    rest = [p for p in on.pairs[2].tolist() if p[1] != top]
    assert len(glob) == 1 and len(rest) >= 1
    assert off.pairs[2].tolist() == sorted(rest) + [[glob[0][0], -1]]


@pytest.mark.parametrize("coeffs", [(1.0, 1.7320508, 2.2360679), (0.3, 0.11, 0.7)])
def test_elevation_unchanged(coeffs):
    f = sf.elevation((7, 6, 5), coeffs)
    on, off = oracle.run(f), oracle.run(f, virtual_max=False)
    for d in range(3):
        assert np.array_equal(on.pairs[d], off.pairs[d])
