"""``torch.autograd.Function`` over the forward (rbp_solve_batch) and the
implicit-KKT backward (rbp_backward) of the library."""
from __future__ import annotations

import torch

from . import _lib
from .api import SegmentBatchGPU


class RBPSolve(torch.autograd.Function):
    """(x0 [N,6], goal [N,3], b_face [F]) -> (P* flat [3*points_total], f* [N]).

    Gradients flow to x0, goal and the shared face offsets b_face (the
    per-instance face gradients are scatter-added into the table).  Instances
    that are not SOLVED contribute zero gradient; ``status`` of the last call
    is kept on the batch object as ``last_status``.

    The library keeps one stored forward state per batch (the last forward
    pass), so a node's backward is only valid while its forward is still the
    batch's last one: a later forward on the same batch (another node, or an
    eager ``solve``) makes the earlier node's backward raise instead of
    differentiating the wrong KKT system.
    """

    @staticmethod
    def forward(ctx, x0, goal, b_face, batch: SegmentBatchGPU, opts=None):
        # a private copy: the caller's options object is left as it was
        o = _lib.SolveOpts.from_buffer_copy(opts) if opts is not None else _lib.default_opts()
        o.store_for_backward = 1
        res = batch.solve(x0.detach().contiguous(), goal.detach().contiguous(),
                          None if b_face is None else b_face.detach().contiguous(), opts=o)
        batch.last_status = res.status
        batch.last_kkt = res.kkt
        ctx.batch = batch
        ctx.generation = batch.forward_generation
        ctx.has_b = b_face is not None
        ctx.mark_non_differentiable(res.status)
        return res.P, res.cost, res.status

    @staticmethod
    def backward(ctx, gP, gcost, _gstatus):
        batch: SegmentBatchGPU = ctx.batch
        if batch.forward_generation != ctx.generation:
            raise RuntimeError("RBPSolve.backward: the batch ran another forward pass after this node's "
                               "forward; its stored KKT state belongs to that later pass")
        gP = None if gP is None else torch.nan_to_num(gP.contiguous(), nan=0.0)
        gcost = None if gcost is None else torch.nan_to_num(gcost.contiguous(), nan=0.0, posinf=0.0, neginf=0.0)
        g = batch.backward(gP, gcost)
        gb = None
        if ctx.has_b:
            gb = torch.zeros(batch.b_face.numel(), dtype=torch.float64, device=batch.device)
            gb.index_add_(0, batch.face_index, g.b_inst)
        return g.x0, g.goal, gb, None, None


def solve(x0, goal, b_face, batch: SegmentBatchGPU, opts=None):
    return RBPSolve.apply(x0, goal, b_face, batch, opts)
