"""Host-side checks of the C-ABI library (no GPU needed): it loads, it
exports every function include/dms.h declares, the binding refuses to run
without it, the batch layout (computed on the host) places disjoint boxes
with a +inf plane between any two, grids are marshalled from 2D and 3D
tensors, and the server admits requests in arrival order within its budget.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "dms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dms_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2206_13932_amd import dms
    names = _declared_functions()
    assert "dms_diagram" in names and "dms_diagram_batch" in names and "dms_scatter_grad" in names
    lib = ctypes.CDLL(dms.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_fails_loudly_without_the_library(monkeypatch):
    from paper_2206_13932_amd import dms
    monkeypatch.setattr(dms, "_lib", None)
    monkeypatch.setattr(dms, "LIB_PATH", os.path.join(ROOT, "no_such_libdms.so"))
    with pytest.raises(ImportError):
        dms.load_library()


@pytest.mark.parametrize("seed", range(6))
def test_batch_layout_boxes_are_disjoint_with_gaps(seed):
    from paper_2206_13932_amd import dms
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 120))
    lo, hi = (2, 40) if seed % 2 else (16, 129)
    shapes = [tuple(int(x) for x in rng.integers(lo, hi, size=3)) for _ in range(n)]
    (X, Y, Z), org = dms.batch_layout(shapes)
    assert X % 16 == 0 and Y % 16 == 0 and Z % 16 == 0
    occ = np.zeros((Z, Y, X), dtype=np.int32)
    for i, (nz, ny, nx) in enumerate(shapes):
        ox, oy, oz = org[i]
        assert ox >= 0 and oy >= 0 and oz >= 0
        assert ox + nx <= X and oy + ny <= Y and oz + nz <= Z
        # the box and the +inf planes that follow it on each axis are its own
        sub = occ[oz:oz + nz + 1, oy:oy + ny + 1, ox:ox + nx + 1]
        assert (sub == 0).all(), i
        sub += 1
    real = sum(a * b * c for a, b, c in shapes)
    assert real <= X * Y * Z


def test_batch_layout_rejects_items_wider_than_the_cross_section():
    from paper_2206_13932_amd import dms
    with pytest.raises(dms.DmsError):
        dms.batch_layout([(10, 10, 64)], cross=(48, 48))
    with pytest.raises(dms.DmsError):
        dms.batch_layout([(1, 10, 10)])


def test_grid_marshalling_of_2d_and_3d_fields():
    import torch
    from paper_2206_13932_amd import dms
    g = dms._grid_of(torch.zeros((4, 5, 6)))
    assert (g.nx, g.ny, g.nz) == (6, 5, 4)
    g = dms._grid_of(torch.zeros((5, 6)))  # [ny, nx]: a 2D grid
    assert (g.nx, g.ny, g.nz) == (6, 5, 1)
    g = dms._grid_of(torch.zeros((1, 5, 6)))
    assert (g.nx, g.ny, g.nz) == (6, 5, 1)
    with pytest.raises(ValueError):
        dms._grid_of(torch.zeros(7))


@pytest.mark.parametrize("budget", [1 << 16, 1 << 18, 1 << 21])
def test_serving_admission_is_fifo_and_fits_the_budget(budget):
    """Host-side admission of the server (no GPU): batches take requests in
    arrival order, and a batch of more than one request has a super grid
    within the vertex budget."""
    import collections
    import threading

    import torch
    from paper_2206_13932_amd import dms, serving
    rng = np.random.default_rng(budget % 97)
    srv = object.__new__(serving.Server)
    srv.cfg = serving.ServerConfig(workers=1, budget_vertices=budget, max_items=32)
    srv.lock = threading.Condition()
    srv.queue = collections.deque()
    shapes = [tuple(int(s) for s in rng.integers(2, 40, size=3)) for _ in range(200)]
    for i, sh in enumerate(shapes):
        srv.queue.append(serving.Request(i, 0.0, torch.zeros(sh)))
    taken = []
    while srv.queue:
        with srv.lock:
            batch = srv._take_batch()
        assert 1 <= len(batch) <= 32
        if len(batch) > 1:
            (X, Y, Z), _ = dms.batch_layout([tuple(r.host_field.shape) for r in batch], srv.cfg.cross,
                                            srv.cfg.z_quantum)
            assert X * Y * Z <= budget
        taken += [r.rid for r in batch]
    assert taken == list(range(len(shapes)))
