"""Differentiable persistence diagrams for topological losses.

A pair's birth (death) value is f at the highest vertex of its birth (death)
simplex in the vertex order (persistence is measured on those values,
Sec. 2.1; the diagram assembly of Sec. 6 reports them). Away from ties the
pairing is locally constant in f, so

    dL/df[v] = sum of dL/d(birth) over the pairs born at v
             + sum of dL/d(death) over the pairs dying at v.

The forward pass is the whole HIP pipeline (dms_diagram); the backward pass
is the library's deterministic scatter (dms_scatter_grad). Contributions are
listed per dimension 0, 1, 2 as all births in pair order, then all finite
deaths in pair order, and each vertex sums its contributions in that order in
float32. The death of an infinite class is the maximum of f, reported as a
value with no vertex: it is treated as a constant.
"""
from __future__ import annotations

import torch

from . import dms


def contribution_list(birth_vertex, death_vertex, grad_birth, grad_death):
    """The canonical (vertex, dL/dvalue) list of the backward pass."""
    verts, grads = [], []
    for d in range(3):
        verts.append(birth_vertex[d])
        grads.append(grad_birth[d])
        fin = death_vertex[d] >= 0
        verts.append(death_vertex[d][fin])
        grads.append(grad_death[d][fin])
    return torch.cat(verts), torch.cat(grads)


class PersistenceFunction(torch.autograd.Function):
    """field -> (birth values D0..D2, death values D0..D2, pairs D0..D2)."""

    @staticmethod
    def forward(ctx, field: torch.Tensor, dms_ctx: dms.Context):
        out = dms_ctx.diagram(field.detach(), with_values=True)
        pairs = [out[d]["pairs"] for d in range(3)]
        bv = [out[d]["birth_vertex"] for d in range(3)]
        dv = [out[d]["death_vertex"] for d in range(3)]
        ctx.save_for_backward(*bv, *dv)
        ctx.nvert = field.numel()
        ctx.shape = field.shape
        ctx.dms_ctx = dms_ctx
        ctx.mark_non_differentiable(*pairs)
        return (*[out[d]["birth_value"] for d in range(3)], *[out[d]["death_value"] for d in range(3)], *pairs)

    @staticmethod
    def backward(ctx, gb0, gb1, gb2, gd0, gd1, gd2, *unused):
        saved = ctx.saved_tensors
        verts, grads = contribution_list(saved[:3], saved[3:], (gb0, gb1, gb2), (gd0, gd1, gd2))
        g = ctx.dms_ctx.scatter_grad(verts, grads, ctx.nvert)
        return g.view(ctx.shape), None


def persistence(field: torch.Tensor, ctx: dms.Context | None = None):
    """Persistence diagrams of a float32 device field [nz, ny, nx] with
    differentiable values: {d: {"pairs", "birth", "death"}} for d = 0, 1, 2.
    The context must outlive the backward pass when one is given."""
    ctx = ctx or dms.Context(field.device.index or 0)
    r = PersistenceFunction.apply(field, ctx)
    return {d: {"pairs": r[6 + d], "birth": r[d], "death": r[3 + d]} for d in range(3)}


def d12_squared_persistence(field: torch.Tensor, ctx: dms.Context | None = None) -> torch.Tensor:
    """The sum over the finite D1 and D2 pairs of (death - birth)^2."""
    p = persistence(field, ctx)
    loss = field.new_zeros(())
    for d in (1, 2):
        fin = p[d]["pairs"][:, 1] >= 0
        loss = loss + ((p[d]["death"] - p[d]["birth"])[fin] ** 2).sum()
    return loss
