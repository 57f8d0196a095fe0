"""torch.autograd.Function over the library's forward and VJP calls.

forward:  p3t_build_tree + p3t_long_force  ->  (acc [n,3], pot [n])
backward: p3t_long_force_vjp with w = dL/dacc, c = dL/dpot  ->  (dL/dpos, dL/dmass)

The backward differentiates the tree force with its lists held fixed.  It
reuses the context's tree when that is still the forward's tree, and rebuilds
it from the saved inputs otherwise (the build is deterministic, so the lists
are the same).  With recompute_lists=True the forward frees the interaction
lists after the force and the backward walks the tree again to recreate them
(for memory pressure; the gradient is the same).
"""
from __future__ import annotations

import torch

from .p3t import P3T


class LongForceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mass, engine: P3T, params: dict, recompute_lists: bool = False):
        pos_d = pos.detach().contiguous()
        mass_d = mass.detach().contiguous()
        engine.build_tree(pos_d, mass_d, **params)
        acc, pot = engine.long_force()
        if recompute_lists:
            engine.release_lists()
        ctx.engine = engine
        ctx.params = dict(params)
        ctx.build_id = engine.build_id
        ctx.save_for_backward(pos_d, mass_d)
        return acc, pot

    @staticmethod
    def backward(ctx, gacc, gpot):
        engine: P3T = ctx.engine
        pos_d, mass_d = ctx.saved_tensors
        if engine.build_id != ctx.build_id:
            engine.build_tree(pos_d, mass_d, **ctx.params)
        w = torch.zeros_like(pos_d) if gacc is None else gacc.contiguous().to(torch.float64)
        c = None if gpot is None else gpot.contiguous().to(torch.float64)
        gpos, gmass = engine.long_force_vjp(w, c)
        return gpos, gmass, None, None, None


def long_force(pos: torch.Tensor, mass: torch.Tensor, engine: P3T, recompute_lists: bool = False,
               **params):
    """Differentiable long-range acceleration and potential."""
    return LongForceFn.apply(pos, mass, engine, params, recompute_lists)
