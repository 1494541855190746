"""Persistent 1-cycle generators of the HIP path (Sec. 8), through the C ABI.

Which cycle a pair gets depends on the order in which concurrent columns were
reduced, so the cycles are not compared with the oracle's edge by edge. What
is unique is compared exactly (one cycle per finite D1 pair, in the order of
the D1 list), and every cycle is checked against the definition by the
full-filtration Z2 check: a cycle, born at the birth edge, homologous to the
boundary of the death triangle through earlier triangles.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synthfields as sf

FIELDS = {
    "noise16": lambda: sf.noise((16, 16, 16), 0),
    "noise_aniso": lambda: sf.noise((5, 9, 7), 3),
    "noise_thin": lambda: sf.noise((2, 2, 9), 4),
    "ties": lambda: np.random.default_rng(6).integers(0, 4, size=(9, 8, 7)).astype(np.float32),
    "smooth20": lambda: sf.gaussians((20, 22, 18), 7, k=8, noise_frac=0.01),
    "cube2": lambda: np.arange(8, dtype=np.float32)[::-1].reshape(2, 2, 2).copy(),
    "noise40": lambda: sf.noise((40, 40, 40), 9),
    "smooth64": lambda: sf.gaussians((64, 64, 64), 9, k=16, noise_frac=0.01),
}


def _ctx():
    import torch
    from paper_2206_13932_amd import dms
    return torch, dms, dms.Context(0)


def _check(name, f, ctx, torch):
    print(f"[generators] case={name} shape={f.shape}", flush=True)
    res = oracle.run(f)
    out = ctx.diagram(torch.from_numpy(f).cuda())
    d1 = out[1].cpu().numpy()
    assert np.array_equal(d1, res.pairs[1]), name
    fin = d1[d1[:, 1] >= 0]
    off, edges = ctx.d1_generators()
    off, edges = off.cpu().numpy(), edges.cpu().numpy()
    assert len(off) == len(fin) + 1 and off[0] == 0 and off[-1] == len(edges), name
    assert (np.diff(off) > 0).all(), name
    for i in range(len(fin)):
        z = edges[off[i]:off[i + 1]]
        assert (np.diff(z) > 0).all(), (name, i)
    st = oracle.bf_check_cycles(res.shape, res.rank, fin, off, edges)
    assert (st == 0).all(), (name, np.bincount(st))
    same = sum(np.array_equal(edges[off[i]:off[i + 1]], res.gen1_edges[res.gen1_off[i]:res.gen1_off[i + 1]])
               for i in range(len(fin)))
    print(f"[generators] {name}: {len(fin)} cycles, {len(edges)} edges, {same} equal to the oracle's", flush=True)


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(FIELDS))
def test_generators_valid(name):
    torch, dms, ctx = _ctx()
    _check(name, FIELDS[name](), ctx, torch)
    ctx.close()


@pytest.mark.gpu
def test_generators_two_fields_one_context():
    """A second field replaces the cycles of the first; calling twice gives
    the same cycles."""
    torch, dms, ctx = _ctx()
    _check("noise12_a", sf.noise((12, 12, 12), 21), ctx, torch)
    _check("noise12_b", sf.noise((12, 13, 11), 22), ctx, torch)
    a = [t.cpu().numpy() for t in ctx.d1_generators()]
    b = [t.cpu().numpy() for t in ctx.d1_generators()]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    ctx.close()


@pytest.mark.gpu
def test_generators_errors():
    torch, dms, ctx = _ctx()
    n, e = ctypes.c_int64(), ctypes.c_int64()
    rc = ctx.lib.dms_d1_generators(ctx.h, None, 0, None, 0, ctypes.byref(n), ctypes.byref(e))
    assert rc == dms.DMS_E_STATE
    f = torch.from_numpy(sf.noise((10, 10, 10), 5)).cuda()
    ctx.gradient(f)
    ctx.pairs_d0_d2()
    rc = ctx.lib.dms_d1_generators(ctx.h, None, 0, None, 0, ctypes.byref(n), ctypes.byref(e))
    assert rc == dms.DMS_E_STATE  # D1 not run yet
    d1 = ctx.pairs_d1().cpu().numpy()
    rc = ctx.lib.dms_d1_generators(ctx.h, None, 0, None, 0, ctypes.byref(n), ctypes.byref(e))
    assert rc == dms.DMS_E_CAPACITY
    assert n.value == int((d1[:, 1] >= 0).sum()) and e.value >= 3 * n.value
    off = torch.empty(n.value + 1, dtype=torch.int64, device="cuda")
    small = torch.empty(max(e.value - 1, 1), dtype=torch.int64, device="cuda")
    rc = ctx.lib.dms_d1_generators(ctx.h, ctypes.c_void_p(off.data_ptr()), off.numel(),
                                   ctypes.c_void_p(small.data_ptr()), e.value - 1, ctypes.byref(n), ctypes.byref(e))
    assert rc == dms.DMS_E_CAPACITY
    rc = ctx.lib.dms_d1_generators(ctx.h, None, 5, None, 0, ctypes.byref(n), ctypes.byref(e))
    assert rc == dms.DMS_E_INVAL
    o2, e2 = ctx.d1_generators()
    assert o2.numel() == n.value + 1 and e2.numel() == e.value
    ctx.close()
