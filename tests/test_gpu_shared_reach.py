"""Shared reachable polytopes (one block per degree serving every edge, as the
paper computes the reachable set once for all edges, Sec. III-A) through the
C ABI.

The shared-table batch reads the same doubles as the batch in which every
instance holds its own copy of its block, in the same order, so forward and
backward outputs must agree bit for bit; a seeded sample is also checked
against the FP64 oracle with the usual tolerances.  Table indices out of
range and a block whose size does not fit the instance's degree are
rejected at build time."""
import numpy as np
import pytest
import torch

from oracle import qp
from tests.parity_helpers import KKT_TOL, compare
from workloads import gen

pytestmark = pytest.mark.gpu


def fwd_bwd(batch, opts=None):
    from paper_2411_13507_amd.api import SegmentBatchGPU
    gb = SegmentBatchGPU(batch)
    d = gb.device
    res = gb.solve(torch.as_tensor(batch.x0, device=d), torch.as_tensor(batch.goal, device=d), opts=opts)
    gbar = torch.as_tensor(np.random.default_rng(5).standard_normal(3 * gb.points_total), device=d)
    g = gb.backward(gbar, torch.ones(batch.n, dtype=torch.float64, device=d))
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in dict(P=res.P, cost=res.cost, status=res.status, kkt=res.kkt,
                                                iters=res.iters, gx0=g.x0, ggoal=g.goal, gb=g.b_inst,
                                                flags=g.flags).items()}
    gb.close()
    return out


def same_bits(a, b):
    return all(np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)) for k in a)


def polish_only():
    from paper_2411_13507_amd import _lib
    o = _lib.default_opts()
    o.admm_iters = 0
    return o


@pytest.mark.parametrize("admm", [True, False], ids=["admm", "polish-only"])
def test_shared_equals_per_instance_50k(gpu_available, admm):
    b = gen.with_shared_reach(gen.generate(1, 50_000))
    print(f"case: 50k edges, one shared block of {b.reach_rows(0)} rows, admm={admm}", flush=True)
    o = None if admm else polish_only()
    shared = fwd_bwd(b, o)
    per = fwd_bwd(b.expanded(), o)
    assert same_bits(shared, per)
    st = shared["status"]
    assert set(np.unique(st).tolist()) <= {qp.SOLVED, qp.INFEASIBLE}
    assert np.all(shared["kkt"][st == qp.SOLVED] <= KKT_TOL)
    assert 0.1 < np.mean(st == qp.SOLVED) < 0.9
    idx = np.random.default_rng(21).choice(b.n, 200, replace=False)
    compare(b, shared["P"], shared["cost"], st, shared["kkt"], idx=idx, label="shared50k")


def test_shared_table_mixed_degrees(gpu_available):
    """Degrees 3-9, one block per degree (48 rows each), against the
    per-instance copy and the oracle."""
    b = gen.with_shared_reach(gen.gen_cfg2(indices=range(700)), r=48)
    assert len(b.reach_off) == 8
    print("case: 700 uneven segments, 7 shared blocks", flush=True)
    shared = fwd_bwd(b)
    assert same_bits(shared, fwd_bwd(b.expanded()))
    compare(b, shared["P"], shared["cost"], shared["status"], shared["kkt"], idx=range(0, 700, 3),
            label="shared-uneven")


def test_shared_table_rejects_bad_index_and_size(gpu_available):
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import SegmentBatchGPU
    import dataclasses
    b = gen.with_shared_reach(gen.gen_cfg2(indices=range(40)), r=16)
    bad = dataclasses.replace(b, reach_idx=b.reach_idx.copy())
    bad.reach_idx[5] = len(b.reach_off) - 1          # one past the table
    with pytest.raises(_lib.RbpError, match="rbp_build_batch"):
        SegmentBatchGPU(bad)
    bad.reach_idx[5] = -1
    with pytest.raises(_lib.RbpError, match="rbp_build_batch"):
        SegmentBatchGPU(bad)
    # an instance pointed at the block of another degree
    wrong = dataclasses.replace(b, reach_idx=b.reach_idx.copy())
    i = int(np.argmax(b.degree != b.degree[0]))
    wrong.reach_idx[i] = b.reach_idx[0]
    with pytest.raises(_lib.RbpError, match="rbp_build_batch"):
        SegmentBatchGPU(wrong)
    SegmentBatchGPU(b).close()
