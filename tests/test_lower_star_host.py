"""The GPU gradient kernel's per-vertex routine, built for the host, against the
oracle on every vertex (CPU only).

`tests/lower_star_host.cpp` compiles the kernel's own lower-star code
(`csrc/lower_star.h`, `csrc/star_tables.h`) for the host and runs it on every
vertex of small grids (ProcessLowerStars, Sec. 2.6). The gradient planes it
writes are decoded by the helpers the GPU tests use and compared, cell by
cell, with the oracle's pairs and critical cells. So a change to the routine
is checked without a GPU, on more vertex orders than the GPU suite runs. The
checks cover:
* both label paths: the sorting network for ranks below 2^28, and the counted
  labels the kernel takes on larger grids (ranks shifted past 2^28 here);
* minimum searches over more levels than a vertex has labels (the lanes of a
  wave pass the largest lower-star size among them);
* the rank sort's comparator network on every input, by the 0-1 principle;
* grids two vertices wide on each axis, where many neighbours are missing.
"""
import ctypes
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synthfields as sf
from tests import helpers as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "lower_star_host.cpp")
CSRC = os.path.join(ROOT, "paper_2206_13932_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found: the kernel's routine cannot be built for the host")
    out = str(tmp_path_factory.mktemp("lshost") / "liblshost.so")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", CSRC, SRC, "-o", out],
                   check=True, capture_output=True)
    L = ctypes.CDLL(out)
    L.ls_host_gradient.restype = ctypes.c_int
    L.ls_host_gradient.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint32,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    return L


def host_gradient(L, shape, rank, packed=True, offset=0, levels_mode=0):
    nz, ny, nx = shape
    r = np.ascontiguousarray(rank, dtype=np.uint32).ravel()
    G = np.empty((26, r.size), dtype=np.uint8)
    crit = np.zeros(4, dtype=np.int64)
    rc = L.ls_host_gradient(nx, ny, nz, r.ctypes.data, offset, int(packed), levels_mode, G.ctypes.data,
                            crit.ctypes.data)
    assert rc == 0, f"host routine check {rc} failed"
    return G, crit


def check_against_oracle(L, shape, rank, **kw):
    G, crit = host_gradient(L, shape, rank, **kw)
    V = int(np.prod(shape))
    recs = oracle.lower_star_sample(shape, rank, np.arange(V, dtype=np.int64))
    cells = recs[:, :, 0].ravel()
    want = recs[:, :, 1].ravel()
    keep = cells != -2
    got = H.decode_cells(shape, G, cells[keep])
    assert np.array_equal(got, want[keep])
    c = [int(((cells[keep] & 3) == d)[want[keep] == -1].sum()) for d in range(4)]
    assert list(crit) == c
    assert crit[0] - crit[1] + crit[2] - crit[3] == 1  # Euler characteristic of a box
    return crit


VARIANTS = [
    dict(packed=True, offset=0, levels_mode=0),
    dict(packed=True, offset=0, levels_mode=1),
    dict(packed=True, offset=0, levels_mode=2),
    dict(packed=True, offset=(1 << 28) - 4096, levels_mode=2),  # the largest ranks of the packed path
    dict(packed=False, offset=0, levels_mode=0),
    dict(packed=False, offset=(1 << 28) + 12345, levels_mode=2),  # counted labels past 2^28
    dict(packed=False, offset=(1 << 32) - 4096, levels_mode=1),
]


@pytest.mark.parametrize("variant", range(len(VARIANTS)))
@pytest.mark.parametrize("shape", [(3, 3, 3), (4, 5, 6), (2, 7, 9), (9, 2, 7), (7, 9, 2), (2, 2, 2), (11, 10, 9)])
def test_random_orders(lib, shape, variant):
    rng = np.random.default_rng(1000 + 17 * variant + shape[0] * 100 + shape[1] * 10 + shape[2])
    V = int(np.prod(shape))
    for _ in range(3):
        rank = rng.permutation(V).astype(np.uint32).reshape(shape)
        check_against_oracle(lib, shape, rank, **VARIANTS[variant])


def test_every_cube_order(lib):
    """All 8! = 40,320 vertex orders of one cube, the label paths and search
    levels taken in turn: each vertex's lower star is every subset of its
    neighbours in the cube that some order gives."""
    shape = (2, 2, 2)
    for i, perm in enumerate(itertools.permutations(range(8))):
        rank = np.array(perm, dtype=np.uint32).reshape(shape)
        check_against_oracle(lib, shape, rank, **VARIANTS[i % len(VARIANTS)])


@pytest.mark.parametrize("seed", range(4))
def test_fields_with_ties_and_smooth_fields(lib, seed):
    """The vertex order of float fields with ties (noise quantised to 16 levels),
    of noise and of a Gaussian mixture, from the oracle's order stage."""
    shape = (12, 13, 14)
    q = np.floor(sf.noise(shape, seed) * 16).astype(np.float32)
    for f in (q, sf.noise(shape, 50 + seed), sf.gaussians(shape, seed, k=6, noise_frac=0.01)):
        rank = oracle.vertex_order(f)
        for variant in (0, 2, 5):
            check_against_oracle(lib, shape, rank, **VARIANTS[variant])


def test_rank_sorting_network_zero_one_principle(lib):
    """The 16-key network behind the packed labels sorts all 2^16 inputs of
    zeros and ones, so by the 0-1 principle it sorts every input."""
    lib.ls_host_sortnet_01.restype = ctypes.c_int
    assert lib.ls_host_sortnet_01() == 0


def test_comparison_catches_a_wrong_order(lib):
    """The comparison is not vacuous: the routine run on ranks with the lowest
    and the highest vertex swapped disagrees with the oracle on the true ranks."""
    rng = np.random.default_rng(3)
    shape = (5, 6, 7)
    rank = rng.permutation(int(np.prod(shape))).astype(np.uint32).reshape(shape)
    check_against_oracle(lib, shape, rank)
    wrong = rank.copy().ravel()
    i, j = int(np.argmin(wrong)), int(np.argmax(wrong))
    wrong[i], wrong[j] = wrong[j], wrong[i]
    G, _ = host_gradient(lib, shape, wrong.reshape(shape))
    V = int(np.prod(shape))
    recs = oracle.lower_star_sample(shape, rank, np.arange(V, dtype=np.int64))
    cells, want = recs[:, :, 0].ravel(), recs[:, :, 1].ravel()
    keep = cells != -2
    assert not np.array_equal(H.decode_cells(shape, G, cells[keep]), want[keep])
