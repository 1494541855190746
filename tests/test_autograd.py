"""Differentiation of the persistence map (loss = sum over the finite D1 and
D2 pairs of (death - birth)^2).

CPU: the reference gradient (oracle pairs, values at the highest vertices)
against float64 central finite differences with eps = 1e-6, recomputing the
diagram of each perturbed field, on every vertex whose order the
perturbation leaves unchanged; the in-order float32 scatter against a loop.
GPU: the HIP backward against the CPU reference, bit for bit, on one 96^3
field (oracle pairs) and on the batch of 64 fields of 96^3 (16 Gaussians and
2% noise; every field against the reference built from the GPU forward's
pairs, three of them against the oracle's pairs); the scatter entry point on its own, with repeats, n = 0 and an
index out of range.
"""
import numpy as np
import pytest

import oracle
import synthfields as sf
from oracle import gradref

EPS = 1e-6


def _order_field(f64):
    """A float32 field whose vertex order is that of f64 (ranks are exact)."""
    flat = f64.ravel()
    order = np.lexsort((np.arange(flat.size), flat))
    rank = np.empty(flat.size, dtype=np.int64)
    rank[order] = np.arange(flat.size)
    return rank.astype(np.float32).reshape(f64.shape), rank


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_finite_differences_match_reference_gradient(seed):
    f32 = sf.gaussians((9, 8, 7), seed, k=4, noise_frac=0.02)
    f = f32.astype(np.float64) + np.random.default_rng(seed).random(f32.shape) * 1e-4  # untied in float64
    of, rank = _order_field(f)
    verts = gradref.pair_vertices(oracle.run(of))
    g = gradref.grad_d12_float64(f, verts)
    assert np.abs(g).max() > 0
    checked = 0
    for v in range(f.size):
        fp, fm = f.copy(), f.copy()
        fp.flat[v] += EPS
        fm.flat[v] -= EPS
        ofp, rp = _order_field(fp)
        ofm, rm = _order_field(fm)
        if not (np.array_equal(rp, rank) and np.array_equal(rm, rank)):
            continue  # a perturbation that reorders vertices: the loss has a kink there
        lp = gradref.loss_d12(fp, gradref.pair_vertices(oracle.run(ofp)))
        lm = gradref.loss_d12(fm, gradref.pair_vertices(oracle.run(ofm)))
        fd = (lp - lm) / (2 * EPS)
        assert abs(fd - g[v]) <= 1e-6 * max(1.0, abs(g[v])), (v, fd, g[v])
        checked += 1
    assert checked >= 0.8 * f.size  # the rest sit within eps of another value


def test_scatter_in_order_matches_loop():
    rng = np.random.default_rng(3)
    vertex = rng.integers(0, 50, size=2000)
    grad = (rng.standard_normal(2000) * 10 ** rng.uniform(-6, 3, 2000)).astype(np.float32)
    a = gradref.scatter_in_order(60, vertex, grad)
    b = gradref.scatter_in_order_loop(60, vertex, grad)
    assert np.array_equal(a, b)
    assert (a[50:] == 0).all()


def _cpu_reference_from_oracle(f):
    """In-order float32 scatter of the loss derivatives from the oracle's
    pairs of f (values at the pairs' highest vertices)."""
    verts = gradref.pair_vertices(oracle.run(f))
    fv = f.ravel()
    vl, gl = [], []
    for d in range(3):
        b, dv = verts[d]
        gd = np.zeros(len(b), np.float32)
        if d in (1, 2):
            fin = dv >= 0
            gd[fin] = np.float32(2.0) * (fv[dv[fin]] - fv[b[fin]])
        vl += [b, dv[dv >= 0]]
        gl += [-gd, gd[dv >= 0]]
    return gradref.scatter_in_order(f.size, np.concatenate(vl), np.concatenate(gl))


def _cpu_reference_from_gpu_outputs(out, nvert):
    """In-order float32 scatter of the loss derivatives, from the values and
    vertices the GPU forward returned."""
    verts, grads = [], []
    for d in range(3):
        b = out[d]["birth_vertex"].cpu().numpy()
        dv = out[d]["death_vertex"].cpu().numpy()
        bval = out[d]["birth_value"].cpu().numpy()
        dval = out[d]["death_value"].cpu().numpy()
        gd = np.zeros(len(b), np.float32)
        if d in (1, 2):
            fin = dv >= 0
            gd[fin] = np.float32(2.0) * (dval[fin] - bval[fin])
        verts += [b, dv[dv >= 0]]
        grads += [-gd, gd[dv >= 0]]
    return gradref.scatter_in_order(nvert, np.concatenate(verts), np.concatenate(grads))


@pytest.mark.gpu
def test_backward_matches_cpu_reference_96():
    import torch
    from paper_2206_13932_amd import autograd, dms
    f = sf.gaussians((96, 96, 96), 100, k=16, noise_frac=0.02)
    print("[autograd] oracle on 96^3", flush=True)
    res = oracle.run(f)
    verts = gradref.pair_vertices(res)
    ctx = dms.Context(0)
    x = torch.from_numpy(f).cuda().requires_grad_(True)
    loss = autograd.d12_squared_persistence(x, ctx)
    loss.backward()
    got = x.grad.cpu().numpy().ravel()
    # reference: the oracle's pairs, float32 values and derivatives, in-order sum
    fv = f.ravel()
    vl, gl = [], []
    for d in range(3):
        b, dv = verts[d]
        gd = np.zeros(len(b), np.float32)
        if d in (1, 2):
            fin = dv >= 0
            gd[fin] = np.float32(2.0) * (fv[dv[fin]] - fv[b[fin]])
        vl += [b, dv[dv >= 0]]
        gl += [-gd, gd[dv >= 0]]
    ref = gradref.scatter_in_order(f.size, np.concatenate(vl), np.concatenate(gl))
    assert np.array_equal(got, ref)
    assert np.isclose(float(loss), gradref.loss_d12(f, verts), rtol=1e-5)
    ctx.close()


@pytest.mark.gpu
def test_backward_batch_64_fields_96():
    import torch
    from paper_2206_13932_amd import autograd, dms
    ctx = dms.Context(0)
    for i in range(64):
        f = sf.gaussians((96, 96, 96), 200 + i, k=16, noise_frac=0.02)
        x = torch.from_numpy(f).cuda().requires_grad_(True)
        loss = autograd.d12_squared_persistence(x, ctx)
        loss.backward()
        g1 = x.grad.clone()
        x.grad = None
        autograd.d12_squared_persistence(x, ctx).backward()
        assert torch.equal(g1, x.grad), i  # deterministic
        out = ctx.diagram(x.detach(), with_values=True)
        ref = _cpu_reference_from_gpu_outputs(out, f.size)
        assert np.array_equal(g1.cpu().numpy().ravel(), ref), i
        if i in (0, 37, 63):  # the whole chain against the oracle's pairs
            print(f"[autograd] field {i}: oracle reference", flush=True)
            assert np.array_equal(g1.cpu().numpy().ravel(), _cpu_reference_from_oracle(f)), i
        if i % 16 == 0:
            print(f"[autograd] field {i} ok", flush=True)
    ctx.close()


@pytest.mark.gpu
def test_scatter_grad_entry_point():
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    rng = np.random.default_rng(5)
    for n, nvert in [(0, 10), (1, 1), (5000, 37), (100000, 1 << 20)]:
        v = rng.integers(0, nvert, size=n)
        g = rng.standard_normal(n).astype(np.float32)
        out = ctx.scatter_grad(torch.from_numpy(v).cuda(), torch.from_numpy(g).cuda(), nvert)
        assert np.array_equal(out.cpu().numpy(), gradref.scatter_in_order(nvert, v, g)), (n, nvert)
    with pytest.raises(dms.DmsError):
        ctx.scatter_grad(torch.tensor([0, 10], device="cuda"), torch.ones(2, device="cuda"), 10)
    ctx.close()
