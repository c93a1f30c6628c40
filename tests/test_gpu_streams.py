"""Grouped launches share the device's three side streams across batches.
Batches of several groups (an uneven segment batch, a path batch of several
lengths) built and used side by side, one destroyed while the others are
still in use, and a batch built after the caller created more streams than
the device has hardware queues: every output must stay bit for bit what the
first solve of the same batch gave."""
import numpy as np
import pytest
import torch

from workloads import gen

pytestmark = pytest.mark.gpu


def _seg_solve(gb, b):
    from paper_2411_13507_amd import _lib
    o = _lib.default_opts()
    o.admm_iters = 0
    o.store_for_backward = 1
    x0 = torch.as_tensor(b.x0, device=gb.device)
    goal = torch.as_tensor(b.goal, device=gb.device)
    r = gb.solve(x0, goal, opts=o)
    gP = torch.as_tensor(np.random.default_rng(2).standard_normal(r.P.numel()), device=gb.device)
    g = gb.backward(gP, torch.ones(b.n, dtype=torch.float64, device=gb.device))
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (r.P, r.cost, r.status, r.kkt, g.x0, g.goal, g.b_inst)]


def _chain_solve(cb, c):
    from paper_2411_13507_amd import _lib
    o = _lib.default_opts()
    o.admm_iters = 0
    r = cb.solve(torch.as_tensor(c.x0, device=cb.device), torch.as_tensor(c.goal, device=cb.device), opts=o)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (r.P, r.cost, r.status, r.kkt, r.iters)]


def _same(a, b, label):
    for x, y in zip(a, b):
        x, y = np.asarray(x), np.asarray(y)
        if x.dtype.kind == "f":
            assert np.array_equal(x.view(np.int64), y.view(np.int64)), label
        else:
            assert np.array_equal(x, y), label


def test_batches_share_side_streams(gpu_available):
    from paper_2411_13507_amd.api import ChainBatchGPU, SegmentBatchGPU
    b = gen.gen_cfg2(indices=range(3000))
    c = gen.gen_cfg3(indices=list(range(96)))
    print(f"case: {b.n} uneven segments and {c.n} paths, side streams shared", flush=True)
    ga = SegmentBatchGPU(b)
    cb = ChainBatchGPU(c)
    ref_a = _seg_solve(ga, b)
    ref_c = _chain_solve(cb, c)
    # a second batch of the same problem, used while the first is alive
    gb2 = SegmentBatchGPU(b)
    _same(_seg_solve(gb2, b), ref_a, "second segment batch")
    _same(_chain_solve(cb, c), ref_c, "path batch, second solve")
    # destroying one batch leaves the shared streams to the others
    ga.close()
    _same(_seg_solve(gb2, b), ref_a, "segment batch after another was destroyed")
    _same(_chain_solve(cb, c), ref_c, "path batch after a segment batch was destroyed")
    # more caller streams than hardware queues, then a new path batch
    keep = [torch.cuda.Stream() for _ in range(6)]
    for s in keep:
        with torch.cuda.stream(s):
            torch.zeros(1, device="cuda").add_(1)
    torch.cuda.synchronize()
    cb2 = ChainBatchGPU(c)
    _same(_chain_solve(cb2, c), ref_c, "path batch built after six more streams")
    cb2.close()
    cb.close()
    gb2.close()
