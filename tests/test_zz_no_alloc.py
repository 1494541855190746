"""The allocation-free scatter (dms_scatter_grad_noalloc), called through the
C ABI, against dms_scatter_grad: the same gradient bit for bit on two calls
in a row, the second with fewer contributions and a smaller field (the
static scratch keeps the first call's contents), plus its error paths."""
import ctypes

import numpy as np
import pytest


def _call(ctx, fn, vertex, grad, out):
    p = ctypes.c_void_p
    return fn(ctx.h, vertex.numel(), p(vertex.data_ptr()), p(grad.data_ptr()), out.numel(), p(out.data_ptr()))


@pytest.mark.gpu
def test_noalloc_scatter_equals_scatter():
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    lib = ctx.lib
    rng = np.random.default_rng(5)
    for step, (n, nvert) in enumerate([(3_000_000, 96 ** 3), (70_001, 40 ** 3)]):
        print(f"[noalloc] call {step}: n={n} nvert={nvert}", flush=True)
        # repeated vertices (runs of several contributions) and untouched ones
        vertex = torch.from_numpy(rng.integers(0, nvert // 2, size=n, dtype=np.int64) * 2).cuda()
        grad = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).cuda()
        ref = torch.full((nvert,), 7.0, device="cuda")
        got = torch.full((nvert,), -3.0, device="cuda")
        assert _call(ctx, lib.dms_scatter_grad, vertex, grad, ref) == dms.DMS_OK
        assert _call(ctx, lib.dms_scatter_grad_noalloc, vertex, grad, got) == dms.DMS_OK
        torch.cuda.synchronize()
        assert torch.equal(got, ref), step
        assert float(got[1::2].abs().max()) == 0.0  # odd vertices: no contribution, written as 0
    # an empty list clears the field
    got = torch.full((10,), 1.0, device="cuda")
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    assert _call(ctx, lib.dms_scatter_grad_noalloc, e, e.float(), got) == dms.DMS_OK
    assert float(got.abs().max()) == 0.0
    ctx.close()


@pytest.mark.gpu
def test_noalloc_scatter_errors():
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    lib = ctx.lib
    # more contributions than the static scratch holds: rejected on the host
    vertex = torch.zeros(8, dtype=torch.int64, device="cuda")
    grad = torch.ones(8, device="cuda")
    out = torch.zeros(16, device="cuda")
    p = ctypes.c_void_p
    rc = lib.dms_scatter_grad_noalloc(ctx.h, dms.NOALLOC_MAX_CONTRIB + 1, p(vertex.data_ptr()), p(grad.data_ptr()),
                                      16, p(out.data_ptr()))
    assert rc == dms.DMS_E_INVAL
    assert b"4194304" in lib.dms_last_error(ctx.h)
    # a vertex outside the field: the device flags it, the call reports it
    vertex[3] = 99
    assert _call(ctx, lib.dms_scatter_grad_noalloc, vertex, grad, out) == dms.DMS_E_INVAL
    # and the next call starts from a clear flag
    vertex[3] = 5
    assert _call(ctx, lib.dms_scatter_grad_noalloc, vertex, grad, out) == dms.DMS_OK
    assert float(out[0]) == 7.0 and float(out[5]) == 1.0
    ctx.close()
