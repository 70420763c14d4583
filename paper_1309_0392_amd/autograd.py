"""torch.autograd wrappers: hierarchization forward, its hand-written adjoint
(transposed hierarchization) kernel backward.

    y = hierarchize(u, levels)                 # one grid
    ys = hierarchize_batch(us, levels_list)    # a combination-grid set, one plan
    y = hierarchize_flat(u, levels_list)       # a set stored back to back in one tensor

All are out of place: hierarchize and hierarchize_flat read the input and write
a new tensor (the library's out-of-place launches); hierarchize_batch clones,
then transforms the clones in place.  The backward of y = H u is
grad_u = H^T grad_y,  computed by the library's adjoint kernels.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import torch

from . import sgh


class Hierarchize(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u: torch.Tensor, levels: Tuple[int, ...]):
        ctx.levels = tuple(int(l) for l in levels)
        u = u.detach().contiguous()
        y = torch.empty_like(u)
        sgh.transform_out(sgh.OP_HIERARCHIZE, u, y, ctx.levels)
        return y

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        gy = grad_y.detach().contiguous()
        g = torch.empty_like(gy)
        sgh.transform_out(sgh.OP_ADJOINT, gy, g, ctx.levels)
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


_FLAT: Dict[tuple, "sgh.FlatPlan"] = {}


def flat_plan(op: int, levels: Tuple[Tuple[int, ...], ...], dtype: torch.dtype, device: torch.device) -> "sgh.FlatPlan":
    """The cached relative plan of a set stored back to back (one per op, level list, dtype, device)."""
    key = (op, levels, dtype, device.index)
    plan = _FLAT.get(key)
    if plan is None:
        with torch.cuda.device(device):
            plan = sgh.FlatPlan(op, levels, sgh.F64 if dtype == torch.float64 else sgh.F32)
        _FLAT[key] = plan
    return plan


class FlatSet:
    """A combination set stored back to back, in list order, in one flat tensor
    (grid i at starts[i]), with the relative plans of its hierarchization and
    of its adjoint built once: a forward and backward then cost two plan
    executions, however many grids the set holds."""

    def __init__(self, levels_list, dtype: torch.dtype = torch.float32, device=None):
        self.levels = tuple(tuple(int(l) for l in lv) for lv in levels_list)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.dtype = dtype
        self.fwd = flat_plan(sgh.OP_HIERARCHIZE, self.levels, dtype, self.device)
        self.adj = flat_plan(sgh.OP_ADJOINT, self.levels, dtype, self.device)
        self.total = self.fwd.total
        self.starts = self.fwd.starts

    def views(self, flat: torch.Tensor) -> List[torch.Tensor]:
        return self.fwd.views(flat)

    def hierarchize(self, u: torch.Tensor) -> torch.Tensor:
        return HierarchizeFlat.apply(u, self)


class HierarchizeFlat(torch.autograd.Function):
    """A combination set held back to back in one flat tensor: forward writes
    the hierarchized set into a new tensor, backward the adjoint of the
    incoming gradient, each as the out-of-place launches of one relative plan
    (no copy, no task-list upload, no synchronization)."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, fs: "FlatSet"):
        ctx.fs = fs
        u = u.detach().contiguous()
        y = torch.empty_like(u)
        fs.fwd.execute_out(u, y)
        return y

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        gy = grad_y.detach().contiguous()
        g = torch.empty_like(gy)
        ctx.fs.adj.execute_out(gy, g)
        return g, None


def hierarchize_flat(u: torch.Tensor, levels_list) -> torch.Tensor:
    """y = H u for a set stored back to back in u; `levels_list` is a list of
    level vectors or a FlatSet (which skips the per-call plan lookup)."""
    fs = levels_list if isinstance(levels_list, FlatSet) else FlatSet(levels_list, u.dtype, u.device)
    return HierarchizeFlat.apply(u, fs)
