"""Reference gradient of persistence-pair values -- TEST INFRASTRUCTURE.

Only tests/ may import this module. A pair's value at birth (death) is f at
the highest vertex, in the vertex order, of its birth (death) simplex
(Sec. 2.1: the lower-star filtration enters a simplex with its highest
vertex). For a loss L of the pair values, dL/df[v] sums dL/d(value) over the
values taken at v. Everything here is plain numpy over the oracle's pairs.
"""
from __future__ import annotations

import numpy as np

from . import OracleResult, simplex_vertices


def pair_vertices(res: OracleResult):
    """Per dimension: (birth vertex int64[n], death vertex int64[n], -1 for an
    infinite class), in the oracle's pair order."""
    out = []
    for d in range(3):
        p = res.pairs[d]
        if p.size == 0:
            out.append((np.zeros(0, np.int64), np.zeros(0, np.int64)))
            continue
        bv = simplex_vertices(res.shape, d, p[:, 0])
        b = bv[np.arange(len(bv)), res.rank[bv].argmax(axis=1)]
        dvert = np.full(len(p), -1, dtype=np.int64)
        fin = p[:, 1] >= 0
        if fin.any():
            dv = simplex_vertices(res.shape, d + 1, p[fin, 1])
            dvert[fin] = dv[np.arange(len(dv)), res.rank[dv].argmax(axis=1)]
        out.append((b.astype(np.int64), dvert))
    return out


def loss_d12(f: np.ndarray, verts) -> float:
    """Sum over the finite D1 and D2 pairs of (death - birth)^2, in float64."""
    x = np.asarray(f, dtype=np.float64).ravel()
    total = 0.0
    for d in (1, 2):
        b, dv = verts[d]
        fin = dv >= 0
        total += float(((x[dv[fin]] - x[b[fin]]) ** 2).sum())
    return total


def grad_d12_float64(f: np.ndarray, verts) -> np.ndarray:
    """dL/df of loss_d12 for a fixed pairing, in float64."""
    x = np.asarray(f, dtype=np.float64).ravel()
    g = np.zeros_like(x)
    for d in (1, 2):
        b, dv = verts[d]
        fin = dv >= 0
        w = 2.0 * (x[dv[fin]] - x[b[fin]])
        np.add.at(g, dv[fin], w)
        np.add.at(g, b[fin], -w)
    return g


def scatter_in_order_loop(nvert: int, vertex: np.ndarray, grad: np.ndarray) -> np.ndarray:
    """out[v] = sum of grad[i] over vertex[i] == v, added in increasing i in
    float32 starting from 0 (a plain loop)."""
    out = np.zeros(nvert, dtype=np.float32)
    g = np.asarray(grad, dtype=np.float32)
    for i, v in enumerate(np.asarray(vertex, dtype=np.int64)):
        out[v] = np.float32(out[v] + g[i])
    return out


def scatter_in_order(nvert: int, vertex: np.ndarray, grad: np.ndarray) -> np.ndarray:
    """The same with numpy's unbuffered add.at (one element at a time, in
    index order, in the array's dtype)."""
    out = np.zeros(nvert, dtype=np.float32)
    np.add.at(out, np.asarray(vertex, dtype=np.int64), np.asarray(grad, dtype=np.float32))
    return out
