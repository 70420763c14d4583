"""torch.autograd wrappers: hierarchization forward, its hand-written adjoint
(transposed hierarchization) kernel backward.

    y = hierarchize(u, levels)                 # one grid
    ys = hierarchize_batch(us, levels_list)    # a combination-grid set, one plan

Both are out of place (the input is cloned, then transformed in place on the
GPU).  The backward of y = H u is  grad_u = H^T grad_y,  computed by the
library's adjoint kernels on a clone of grad_y.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import torch

from . import sgh


class Hierarchize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, levels: Tuple[int, ...]):
        ctx.levels = tuple(int(l) for l in levels)
        y = u.detach().contiguous().clone()
        sgh.hierarchize(y, ctx.levels)
        return y

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        g = grad_y.detach().contiguous().clone()
        sgh.hierarchize_adjoint(g, ctx.levels)
        return g, None


def hierarchize(u: torch.Tensor, levels: Sequence[int]) -> torch.Tensor:
    return Hierarchize.apply(u, tuple(int(l) for l in levels))


_PLANS: Dict[tuple, "sgh.Plan"] = {}


def _plan(op: int, levels: List[Tuple[int, ...]], tensors) -> "sgh.Plan":
    key = (op, tuple(levels), tuple(t.dtype for t in tensors), tensors[0].device.index)
    plan = _PLANS.get(key)
    if plan is None:
        plan = sgh.Plan(op, tensors, levels, graph=True)
        _PLANS[key] = plan
    else:
        plan.set_data(tensors)
    return plan


class HierarchizeBatch(torch.autograd.Function):
    """All grids of a combination set in one batched plan (one launch for the grids that fit on chip)."""

    @staticmethod
    def forward(ctx, levels: Tuple[Tuple[int, ...], ...], *us: torch.Tensor):
        ctx.levels = list(levels)
        ctx.meta = [(u.shape, u.dtype, u.device) for u in us]
        ys = [u.detach().contiguous().clone() for u in us]
        _plan(sgh.OP_HIERARCHIZE, ctx.levels, ys).execute()
        return tuple(ys)

    @staticmethod
    def backward(ctx, *grads: torch.Tensor):
        gs = []
        for g, (shape, dtype, device) in zip(grads, ctx.meta):
            if g is None:  # output not used by the loss
                gs.append(torch.zeros(shape, dtype=dtype, device=device))
            else:
                gs.append(g.detach().contiguous().clone())
        _plan(sgh.OP_ADJOINT, ctx.levels, gs).execute()
        return (None,) + tuple(gs)


def hierarchize_batch(us: Sequence[torch.Tensor], levels_list) -> List[torch.Tensor]:
    levels = tuple(tuple(int(l) for l in lv) for lv in levels_list)
    return list(HierarchizeBatch.apply(levels, *us))
