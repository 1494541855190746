"""Shared test helpers: simplex id arithmetic in numpy (written for the tests,
independent of both the oracle's C++ and the HIP library)."""
from __future__ import annotations

import numpy as np

NTYPES = (1, 7, 12, 6)
STEPS = {
    1: [[1], [2], [3], [4], [5], [6], [7]],
    2: [[1, 2], [1, 4], [1, 6], [2, 1], [2, 4], [2, 5], [3, 4], [4, 1], [4, 2], [4, 3],
        [5, 2], [6, 1]],
    3: [[1, 2, 4], [1, 4, 2], [2, 1, 4], [2, 4, 1], [4, 1, 2], [4, 2, 1]],
}


def coords(shape, v):
    nz, ny, nx = shape
    v = np.asarray(v, dtype=np.int64)
    return np.stack([v % nx, (v // nx) % ny, v // (nx * ny)], axis=-1)


def vertices(shape, dim, ids):
    """(n, dim+1) vertex ids in chain order; -1 rows for ids outside the grid."""
    nz, ny, nx = shape
    ids = np.asarray(ids, dtype=np.int64)
    if dim == 0:
        return ids[:, None].copy()
    anchor, typ = ids // NTYPES[dim], ids % NTYPES[dim]
    c = coords(shape, anchor)
    out = np.empty((ids.size, dim + 1), dtype=np.int64)
    out[:, 0] = anchor
    ok = anchor < nx * ny * nz
    table = np.array(STEPS[dim])
    n = np.array([nx, ny, nz])
    for s in range(dim):
        m = table[typ, s]
        for a in range(3):
            c[:, a] += (m >> a) & 1
        ok &= (c < n).all(axis=1)
        out[:, s + 1] = c[:, 0] + nx * (c[:, 1] + ny * c[:, 2])
    out[~ok] = -1
    return out


def ids_from_vertices(shape, dim, verts):
    """Inverse of vertices(): rows of ascending vertex ids -> simplex ids."""
    verts = np.asarray(verts, dtype=np.int64)
    if dim == 0:
        return verts[:, 0].copy()
    lut = np.full(8 ** dim, -1, dtype=np.int64)
    for t, st in enumerate(STEPS[dim]):
        lut[sum(m << (3 * i) for i, m in enumerate(st))] = t
    c = coords(shape, verts)
    code = np.zeros(len(verts), dtype=np.int64)
    for s in range(dim):
        d = c[:, s + 1] - c[:, s]
        assert ((d == 0) | (d == 1)).all()
        code |= (d[:, 0] | (d[:, 1] << 1) | (d[:, 2] << 2)) << (3 * s)
    typ = lut[code]
    assert (typ >= 0).all()
    return verts[:, 0] * NTYPES[dim] + typ


def facets(shape, dim, ids):
    """(n, dim+1) facet ids (dropping vertex 0, 1, ...)."""
    vs = vertices(shape, dim, ids)
    cols = []
    for drop in range(dim + 1):
        keep = [i for i in range(dim + 1) if i != drop]
        cols.append(ids_from_vertices(shape, dim - 1, vs[:, keep]))
    return np.stack(cols, axis=1)


def existing(shape, dim):
    nz, ny, nx = shape
    ids = np.arange(nx * ny * nz * NTYPES[dim], dtype=np.int64)
    ok = vertices(shape, dim, ids)[:, 0] >= 0
    return ids[ok]


def as_set(rows):
    return sorted(map(tuple, np.asarray(rows).tolist()))


PLANE_BASE = (0, 1, 8, 20)


def decode_gradient(shape, G):
    """GPU gradient byte planes (26*V bytes) -> tagged partner ids per
    dimension, in the oracle's convention (id*4+dim, -1 critical, -2 absent)."""
    nz, ny, nx = shape
    V = nx * ny * nz
    G = np.asarray(G, dtype=np.uint8).reshape(26, V)
    out = []
    for dim in range(4):
        res = np.empty(NTYPES[dim] * V, dtype=np.int64)
        for t in range(NTYPES[dim]):
            code = G[PLANE_BASE[dim] + t].astype(np.int64)
            ids = np.arange(V, dtype=np.int64) * NTYPES[dim] + t
            r = np.full(V, -3, dtype=np.int64)
            r[code == 0xFF] = -1
            r[code == 0xFE] = -2
            up = code < 27
            if up.any():
                vs = vertices(shape, dim, ids[up])
                a = coords(shape, vs[:, 0])
                c = code[up]
                w = a + np.stack([c % 3 - 1, (c // 3) % 3 - 1, c // 9 - 1], axis=1)
                wid = w[:, 0] + nx * (w[:, 1] + ny * w[:, 2])
                allv = np.sort(np.concatenate([vs, wid[:, None]], axis=1), axis=1)
                r[up] = ids_from_vertices(shape, dim + 1, allv) * 4 + dim + 1
            dn = (code >= 0x80) & (code < 0x84)
            if dn.any():
                vs = vertices(shape, dim, ids[dn])
                i = code[dn] & 3
                keep = np.ones(vs.shape, dtype=bool)
                keep[np.arange(len(vs)), i] = False
                sub = vs[keep].reshape(len(vs), dim)
                r[dn] = ids_from_vertices(shape, dim - 1, sub) * 4 + dim - 1
            res[t::NTYPES[dim]] = r
        out.append(res)
    return out


def decode_cells(shape, G, tagged):
    """Partners (tagged id*4+dim, -1 critical, -2 absent) of the tagged cells,
    read from the GPU gradient planes G (26, V) uint8."""
    nz, ny, nx = shape
    tagged = np.asarray(tagged, dtype=np.int64)
    out = np.full(tagged.size, -3, dtype=np.int64)
    for dim in range(4):
        sel = np.nonzero((tagged & 3) == dim)[0]
        if sel.size == 0:
            continue
        ids = tagged[sel] >> 2
        anchor, typ = ids // NTYPES[dim], ids % NTYPES[dim]
        code = G[PLANE_BASE[dim] + typ, anchor].astype(np.int64)
        r = np.full(sel.size, -3, dtype=np.int64)
        r[code == 0xFF] = -1
        r[code == 0xFE] = -2
        up = code < 27
        if up.any():
            vs = vertices(shape, dim, ids[up])
            a = coords(shape, vs[:, 0])
            c = code[up]
            w = a + np.stack([c % 3 - 1, (c // 3) % 3 - 1, c // 9 - 1], axis=1)
            wid = w[:, 0] + nx * (w[:, 1] + ny * w[:, 2])
            allv = np.sort(np.concatenate([vs, wid[:, None]], axis=1), axis=1)
            r[up] = ids_from_vertices(shape, dim + 1, allv) * 4 + dim + 1
        dn = (code >= 0x80) & (code < 0x84)
        if dn.any():
            vs = vertices(shape, dim, ids[dn])
            i = code[dn] & 3
            keep = np.ones(vs.shape, dtype=bool)
            keep[np.arange(len(vs)), i] = False
            sub = vs[keep].reshape(len(vs), dim)
            r[dn] = ids_from_vertices(shape, dim - 1, sub) * 4 + dim - 1
        out[sel] = r
    return out
