"""2D grids (nz = 1) on the HIP path, through the C ABI, against the oracle.

On a 2D grid D1 comes from the stable sets of the 1-saddles and the dual
union-find (Sec. 3, 5.2), not from the sandwich. Everything integer must be
bit-identical: vertex order, gradient planes, critical sets, D0 arcs, D0, D1
and the (empty) D2.
"""
import ctypes

import numpy as np
import pytest

import synthfields as sf
from tests.test_gpu_parity import _check_all, _gpu_ctx

FIELDS_2D = {
    "noise_16": lambda: sf.noise((1, 16, 16), 0),
    "noise_33x17": lambda: sf.noise((1, 33, 17), 1),
    "thin": lambda: sf.noise((1, 2, 40), 2),
    "square": lambda: np.arange(4, dtype=np.float32)[::-1].reshape(1, 2, 2).copy(),
    "ties": lambda: np.random.default_rng(6).integers(0, 4, size=(1, 12, 11)).astype(np.float32),
    "smooth_48x40": lambda: sf.gaussians((1, 48, 40), 3, k=8, noise_frac=0.01),
    "noise_300x257": lambda: sf.noise((1, 300, 257), 4),
    "smooth_512": lambda: sf.gaussians((1, 512, 512), 5, k=32, noise_frac=0.01),
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(FIELDS_2D))
def test_parity_2d(name):
    torch, dms, ctx = _gpu_ctx()
    res = _check_all(name, FIELDS_2D[name](), ctx, torch, dms)
    assert len(res.pairs[2]) == 0
    ctx.close()


@pytest.mark.gpu
def test_2d_field_given_as_a_matrix():
    """A [ny, nx] tensor is the same 2D grid as [1, ny, nx]."""
    torch, dms, ctx = _gpu_ctx()
    f = sf.noise((1, 18, 23), 11)
    a = ctx.diagram(torch.from_numpy(f).cuda())
    b = ctx.diagram(torch.from_numpy(f[0].copy()).cuda())
    for d in range(3):
        assert np.array_equal(a[d].cpu().numpy(), b[d].cpu().numpy())
    ctx.close()


@pytest.mark.gpu
def test_2d_then_3d_in_one_context():
    torch, dms, ctx = _gpu_ctx()
    _check_all("noise_2d", sf.noise((1, 20, 24), 7), ctx, torch, dms)
    _check_all("noise_3d", sf.noise((8, 9, 10), 8), ctx, torch, dms)
    _check_all("noise_2d_again", sf.noise((1, 24, 20), 9), ctx, torch, dms)
    ctx.close()


@pytest.mark.gpu
def test_2d_has_no_sandwich_generators():
    torch, dms, ctx = _gpu_ctx()
    ctx.diagram(torch.from_numpy(sf.noise((1, 12, 12), 3)).cuda())
    n, e = ctypes.c_int64(), ctypes.c_int64()
    rc = ctx.lib.dms_d1_generators(ctx.h, None, 0, None, 0, ctypes.byref(n), ctypes.byref(e))
    assert rc == dms.DMS_E_STATE
    with pytest.raises(dms.DmsError) as err:
        ctx.gradient(torch.zeros((1, 1, 5), device="cuda"))
    assert err.value.code == dms.DMS_E_INVAL
    ctx.close()
