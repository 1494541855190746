"""CPU oracle of the Discrete Morse Sandwich pipeline -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its binding) never imports it and shares no code with it.

Two native libraries are built from the C++ sources next to this file with
the host compiler:

* ``liboracle.so``     -- the sequential pipeline (dms_oracle.cpp).
* ``libbruteforce.so`` -- full-filtration Z2 reduction and lower-link Betti
  numbers (bruteforce.cpp), which pin the oracle to the definitions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS = {
    "oracle": ("dms_oracle.cpp", "liboracle.so"),
    "bruteforce": ("bruteforce.cpp", "libbruteforce.so"),
}
_loaded = {}

ORC_RANK, ORC_PARTNER0, ORC_CRIT0 = 0, 1, 5
ORC_D0, ORC_D1, ORC_D2, ORC_ARCS0, ORC_ARCS2, ORC_TIMES = 9, 10, 11, 12, 13, 14
ORC_GEN1_OFF, ORC_GEN1_EDGES, ORC_D1_ADDS = 15, 16, 17
NTYPES = (1, 7, 12, 6)


def build(force: bool = True) -> None:
    """Compile both oracle libraries with g++ (host code only)."""
    for src, lib in _LIBS.values():
        out = os.path.join(_HERE, lib)
        if not force and os.path.exists(out):
            continue
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", out + ".tmp",
               os.path.join(_HERE, src)]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)


def _lib(name: str) -> ctypes.CDLL:
    if name in _loaded:
        return _loaded[name]
    path = os.path.join(_HERE, _LIBS[name][1])
    if not os.path.exists(path):
        build(force=False)
    lib = ctypes.CDLL(path)
    i64, p = ctypes.c_int64, ctypes.c_void_p
    if name == "oracle":
        lib.orc_run.argtypes = [i64, i64, i64, p, ctypes.POINTER(p), ctypes.c_char_p, ctypes.c_int]
        lib.orc_run.restype = ctypes.c_int
        lib.orc_run_opts.argtypes = [i64, i64, i64, p, ctypes.c_int, ctypes.POINTER(p), ctypes.c_char_p, ctypes.c_int]
        lib.orc_run_opts.restype = ctypes.c_int
        lib.orc_size.argtypes = [p, ctypes.c_int]
        lib.orc_size.restype = i64
        lib.orc_copy.argtypes = [p, ctypes.c_int, p]
        lib.orc_free.argtypes = [p]
        lib.orc_vertex_order.argtypes = [i64, p, p]
        lib.orc_vertex_order.restype = ctypes.c_int
        lib.orc_lower_star_sample.argtypes = [i64, i64, i64, p, i64, p, p]
        lib.orc_lower_star_sample.restype = ctypes.c_int
        lib.orc_time_gradient.argtypes = [i64, i64, i64, p, i64]
        lib.orc_time_gradient.restype = ctypes.c_double
        lib.orc_time_gradient_omp.argtypes = [i64, i64, i64, p, i64, ctypes.POINTER(ctypes.c_int32)]
        lib.orc_time_gradient_omp.restype = ctypes.c_double
    else:
        lib.bf_counts.argtypes = [i64, i64, i64, p]
        lib.bf_counts.restype = i64
        lib.bf_diagram.argtypes = [i64, i64, i64, p, p, i64, p, i64, p]
        lib.bf_diagram.restype = i64
        lib.bf_lower_link_betti.argtypes = [i64, i64, i64, p, p]
        lib.bf_d0_kruskal.argtypes = [i64, i64, i64, p, p, i64]
        lib.bf_d0_kruskal.restype = i64
        lib.bf_d2_dual.argtypes = [i64, i64, i64, p, p, i64]
        lib.bf_d2_dual.restype = i64
    _loaded[name] = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleResult:
    """Everything the oracle computed for one field."""

    def __init__(self, shape, handle):
        lib = _lib("oracle")
        self.shape = shape

        def get(what, dtype, width=1):
            n = lib.orc_size(handle, what)
            a = np.empty(n * width, dtype=dtype)
            if n:
                lib.orc_copy(handle, what, _ptr(a))
            return a.reshape(n, width) if width > 1 else a

        self.rank = get(ORC_RANK, np.uint32)
        self.partner = [get(ORC_PARTNER0 + d, np.int64) for d in range(4)]
        self.crit = [get(ORC_CRIT0 + d, np.int64) for d in range(4)]
        self.pairs = [get(ORC_D0, np.int64, 2), get(ORC_D1, np.int64, 2), get(ORC_D2, np.int64, 2)]
        self.arcs0 = get(ORC_ARCS0, np.int64, 3)
        self.arcs2 = get(ORC_ARCS2, np.int64, 3)
        self.times = get(ORC_TIMES, np.float64)
        # persistent 1-cycle generators (Sec. 8): for the i-th finite D1 pair,
        # gen1_edges[gen1_off[i]:gen1_off[i + 1]] (edge ids, ascending)
        self.gen1_off = get(ORC_GEN1_OFF, np.int64)
        self.gen1_edges = get(ORC_GEN1_EDGES, np.int64)
        # D1 steps that added an earlier 2-saddle's (cached or own) boundary
        self.d1_adds = int(get(ORC_D1_ADDS, np.int64)[0])


def run(field: np.ndarray, sandwich: bool = True, virtual_max: bool = True, cache: bool = True) -> OracleResult:
    """Run the whole oracle pipeline on a float32 field shaped [nz, ny, nx].
    sandwich=False: the ablation of Sec. 3, D1 over every critical triangle
    instead of those D2 left unpaired (the diagrams must not change); defined
    with the virtual maximum only (without it the dual union-find's D2 is not
    the plain reduction's).
    cache=False: the ablation of Sec. 4.1(b), an earlier 2-saddle's own
    boundary added and reduced again instead of its cached one (the diagrams
    must not change; the work can grow steeply).
    virtual_max=False: the optional boundary adjustment of Sec. 5.2 is off
    (the outside is no node of the dual union-find; App. A)."""
    f = np.ascontiguousarray(field, dtype=np.float32)
    nz, ny, nx = f.shape
    lib = _lib("oracle")
    h = ctypes.c_void_p()
    err = ctypes.create_string_buffer(512)
    flags = (0 if sandwich else 1) | (0 if virtual_max else 2) | (0 if cache else 4)
    rc = lib.orc_run_opts(nx, ny, nz, _ptr(f), flags, ctypes.byref(h), err, 512)
    if rc != 0:
        raise ValueError(err.value.decode())
    try:
        return OracleResult((nz, ny, nx), h)
    finally:
        lib.orc_free(h)


def vertex_order(field: np.ndarray) -> np.ndarray:
    f = np.ascontiguousarray(field, dtype=np.float32).ravel()
    r = np.empty(f.size, dtype=np.uint32)
    if _lib("oracle").orc_vertex_order(f.size, _ptr(f), _ptr(r)) != 0:
        raise ValueError("NaN in the scalar field")
    return r


def lower_star_sample(shape, rank: np.ndarray, verts: np.ndarray) -> np.ndarray:
    """(n, 75, 2) records (cell id*4+dim, partner id*4+dim | -1), padded with -2."""
    nz, ny, nx = shape
    v = np.ascontiguousarray(verts, dtype=np.int64)
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    out = np.empty((v.size, 75, 2), dtype=np.int64)
    if _lib("oracle").orc_lower_star_sample(nx, ny, nz, _ptr(r), v.size, _ptr(v), _ptr(out)) != 0:
        raise RuntimeError("oracle lower-star sample failed")
    return out


def time_gradient(shape, rank: np.ndarray, n_verts: int) -> float:
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    return float(_lib("oracle").orc_time_gradient(nx, ny, nz, _ptr(r), n_verts))


def time_gradient_omp(shape, rank: np.ndarray, n_verts: int):
    """(seconds, threads): the gradient stage over the first n_verts
    vertices with the lower stars shared among OpenMP threads."""
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    th = ctypes.c_int32(0)
    dt = float(_lib("oracle").orc_time_gradient_omp(nx, ny, nz, _ptr(r), n_verts, ctypes.byref(th)))
    return dt, int(th.value)


# ------------------------------------------------------------ brute force --

def bf_counts(shape):
    nz, ny, nx = shape
    c = np.zeros(4, dtype=np.int64)
    _lib("bruteforce").bf_counts(nx, ny, nz, _ptr(c))
    return c


def bf_diagram(shape, rank: np.ndarray):
    """Full-filtration reduction: (pairs (n,3) of (dim, birth rank, death
    rank) with positive persistence, essential (m,2) of (dim, birth rank))."""
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    lib = _lib("bruteforce")
    cap = 8 * nx * ny * nz + 64
    pairs = np.empty((cap, 3), dtype=np.int64)
    ess = np.empty((64, 2), dtype=np.int64)
    n_ess = ctypes.c_int64()
    m = lib.bf_diagram(nx, ny, nz, _ptr(r), _ptr(pairs), cap, _ptr(ess), 64, ctypes.byref(n_ess))
    return pairs[:m].copy(), ess[: min(n_ess.value, 64)].copy()


def bf_d0_kruskal(shape, rank: np.ndarray) -> np.ndarray:
    """D0 of the lexicographic filtration from Kruskal's union-find over all
    edges: (birth rank, death rank) pairs with positive persistence, sorted."""
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    cap = nx * ny * nz
    out = np.empty((cap, 2), dtype=np.int64)
    m = _lib("bruteforce").bf_d0_kruskal(nx, ny, nz, _ptr(r), _ptr(out), cap)
    return out[:m].copy()


def bf_d2_dual(shape, rank: np.ndarray) -> np.ndarray:
    """D2 of the lexicographic filtration from the dual union-find over every
    triangle and tetrahedron, with the outside as the oldest node:
    (birth rank, death rank) pairs with positive persistence, sorted."""
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    cap = nx * ny * nz + 16  # at most one maximum per lower star
    out = np.empty((cap, 2), dtype=np.int64)
    m = _lib("bruteforce").bf_d2_dual(nx, ny, nz, _ptr(r), _ptr(out), cap)
    return out[:m].copy()


def bf_check_cycles(shape, rank: np.ndarray, pairs1: np.ndarray, off: np.ndarray, edges: np.ndarray) -> np.ndarray:
    """Check persistent 1-cycle generators against their definition over the
    whole filtration: pairs1 (n, 2) finite D1 pairs (edge id, triangle id),
    generator i = edges[off[i]:off[i + 1]] (edge ids). Returns a status per
    pair (0 = valid; see bf_check_cycles in bruteforce.cpp)."""
    nz, ny, nx = shape
    pairs1 = np.asarray(pairs1, dtype=np.int64).reshape(-1, 2)
    n = len(pairs1)
    tv = np.ascontiguousarray(simplex_vertices(shape, 1, pairs1[:, 0]), dtype=np.int64)
    sv = np.ascontiguousarray(simplex_vertices(shape, 2, pairs1[:, 1]), dtype=np.int64)
    ev = np.ascontiguousarray(simplex_vertices(shape, 1, np.asarray(edges, dtype=np.int64)), dtype=np.int64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    status = np.zeros(n, dtype=np.int32)
    if n:
        _lib("bruteforce").bf_check_cycles(nx, ny, nz, _ptr(r), n, _ptr(tv), _ptr(sv), _ptr(off), _ptr(ev),
                                           _ptr(status))
    return status


def bf_lower_link_betti(shape, rank: np.ndarray) -> np.ndarray:
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32)
    out = np.empty((nx * ny * nz, 4), dtype=np.int32)
    _lib("bruteforce").bf_lower_link_betti(nx, ny, nz, _ptr(r), _ptr(out))
    return out


# -------------------------------------------------- order-space mapping --

def simplex_vertices(shape, dim: int, ids: np.ndarray) -> np.ndarray:
    """Vertex ids (n, dim+1) of simplices given by the id scheme. Written
    here for the order-space comparison; the C++ side has its own."""
    steps = {
        1: [[1], [2], [3], [4], [5], [6], [7]],
        2: [[1, 2], [1, 4], [1, 6], [2, 1], [2, 4], [2, 5], [3, 4], [4, 1], [4, 2], [4, 3],
            [5, 2], [6, 1]],
        3: [[1, 2, 4], [1, 4, 2], [2, 1, 4], [2, 4, 1], [4, 1, 2], [4, 2, 1]],
    }
    nz, ny, nx = shape
    ids = np.asarray(ids, dtype=np.int64)
    if dim == 0:
        return ids[:, None]
    anchor, typ = ids // NTYPES[dim], ids % NTYPES[dim]
    off = {1: 1, 2: nx, 4: nx * ny}
    out = np.empty((ids.size, dim + 1), dtype=np.int64)
    out[:, 0] = anchor
    cur = anchor.copy()
    table = np.array(steps[dim])
    for s in range(dim):
        m = table[typ, s]
        delta = np.zeros_like(cur)
        for bit, o in off.items():
            delta += np.where(m & bit, o, 0)
        cur = cur + delta
        out[:, s + 1] = cur
    return out


def max_vertex_rank(shape, rank: np.ndarray, dim: int, ids: np.ndarray) -> np.ndarray:
    vs = simplex_vertices(shape, dim, ids)
    return rank[vs].max(axis=1).astype(np.int64)


def order_space(res: OracleResult):
    """Map oracle pairs to (dim, birth rank, death rank), dropping pairs of
    zero persistence, plus essential (dim, birth rank)."""
    shape, rank = res.shape, res.rank
    fin, ess = [], []
    for d in range(3):
        p = res.pairs[d]
        if p.size == 0:
            continue
        e = p[:, 1] < 0
        if e.any():
            b = max_vertex_rank(shape, rank, d, p[e, 0])
            ess += [(d, int(x)) for x in b]
        q = p[~e]
        if q.size:
            b = max_vertex_rank(shape, rank, d, q[:, 0])
            dd = max_vertex_rank(shape, rank, d + 1, q[:, 1])
            keep = b != dd
            fin += [(d, int(x), int(y)) for x, y in zip(b[keep], dd[keep])]
    return sorted(fin), sorted(ess)
