"""Host-side logic of the autograd node (no GPU): the stored-state guard and
the options copy.  A stand-in batch object replaces the library calls."""
import types

import pytest
import torch

from paper_2411_13507_amd import _lib
from paper_2411_13507_amd.torch_fn import RBPSolve


class _StubBatch:
    """Mimics SegmentBatchGPU's Python surface: solve() bumps the forward
    generation like the real binding; backward() returns zero gradients."""

    def __init__(self, n=3, npts=8, nfaces=5):
        self.N, self.points_total = n, n * npts
        self.forward_generation = 0
        self.device = torch.device("cpu")
        self.b_face = torch.zeros(nfaces, dtype=torch.float64)
        self.face_index = torch.arange(nfaces, dtype=torch.int64)
        self.seen_opts = []

    def solve(self, x0, goal, b_face=None, opts=None):
        self.forward_generation += 1
        self.seen_opts.append(opts)
        n = self.N
        return types.SimpleNamespace(P=(x0.sum() * torch.ones(3 * self.points_total, dtype=torch.float64)),
                                     cost=torch.zeros(n, dtype=torch.float64),
                                     status=torch.zeros(n, dtype=torch.int32),
                                     kkt=torch.zeros(n, dtype=torch.float64))

    def backward(self, gP, gcost):
        n = self.N
        return types.SimpleNamespace(x0=torch.ones(n, 6, dtype=torch.float64),
                                     goal=torch.ones(n, 3, dtype=torch.float64),
                                     b_inst=torch.ones(self.b_face.numel(), dtype=torch.float64))


def _inputs(b):
    x0 = torch.zeros(b.N, 6, dtype=torch.float64, requires_grad=True)
    goal = torch.zeros(b.N, 3, dtype=torch.float64, requires_grad=True)
    return x0, goal


def test_backward_of_latest_forward_runs():
    b = _StubBatch()
    x0, goal = _inputs(b)
    P, cost, _ = RBPSolve.apply(x0, goal, None, b, None)
    (P.sum() + cost.sum()).backward()
    assert torch.equal(x0.grad, torch.ones_like(x0))


def test_backward_after_a_later_forward_raises():
    b = _StubBatch()
    x0, goal = _inputs(b)
    P1, c1, _ = RBPSolve.apply(x0, goal, None, b, None)
    P2, c2, _ = RBPSolve.apply(x0, goal, None, b, None)
    with pytest.raises(RuntimeError, match="another forward pass"):
        (P1.sum() + c1.sum()).backward(retain_graph=True)
    # the later node is still the batch's stored forward
    (P2.sum() + c2.sum()).backward()


def test_eager_solve_between_forward_and_backward_raises():
    b = _StubBatch()
    x0, goal = _inputs(b)
    P, c, _ = RBPSolve.apply(x0, goal, None, b, None)
    b.solve(x0.detach(), goal.detach())
    with pytest.raises(RuntimeError, match="another forward pass"):
        P.sum().backward()


def test_caller_options_are_not_modified():
    b = _StubBatch()
    x0, goal = _inputs(b)
    o = _lib.default_opts()
    o.store_for_backward = 0
    o.admm_iters = 3
    RBPSolve.apply(x0, goal, None, b, o)
    assert o.store_for_backward == 0
    used = b.seen_opts[-1]
    assert used is not o and used.store_for_backward == 1 and used.admm_iters == 3
