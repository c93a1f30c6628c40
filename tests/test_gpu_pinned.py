"""Pinned start velocity (the full-state start of Lemma 1: the curve leaves
P_0 with derivative x0[3:6]) through the C ABI, against the FP64 oracle.

Forward: the usual tolerances (status bit-exact where the oracle certifies
it, cost 1e-6 relative, P* 1e-6, KKT residual <= 1e-6) on seeded subsets of
the cluttered and uneven batches, the full 50,000 edges sampled (every
instance by properties: b'(0) = x0[3:6], statuses, residuals) and a start
speed above vmax.  Backward: gradients against the oracle's where the
oracle certifies that they are well defined, 1e-4 relative, including
d/d vel(x0), which only the pin rows carry."""
import numpy as np
import pytest
import torch

from oracle import qp, segment
from tests.parity_helpers import GRAD_RTOL, KKT_TOL, compare
from workloads import gen

pytestmark = pytest.mark.gpu


def solve(batch, opts=None):
    from paper_2411_13507_amd.api import SegmentBatchGPU
    gb = SegmentBatchGPU(batch)
    d = gb.device
    res = gb.solve(torch.as_tensor(batch.x0, device=d), torch.as_tensor(batch.goal, device=d), opts=opts)
    torch.cuda.synchronize()
    return gb, {k: getattr(res, k).cpu().numpy() for k in ("P", "cost", "status", "kkt", "iters")}


def polish_only():
    from paper_2411_13507_amd import _lib
    o = _lib.default_opts()
    o.admm_iters = 0
    return o


def start_velocity(batch, P):
    pt = np.concatenate([[0], np.cumsum(batch.degree.astype(np.int64) + 1)])
    v = np.empty((batch.n, 3))
    for i in range(batch.n):
        Pi = P[3 * pt[i]:3 * pt[i + 1]].reshape(-1, 3)
        v[i] = batch.degree[i] / batch.T[i] * (Pi[1] - Pi[0])
    return v


@pytest.mark.parametrize("admm", [True, False], ids=["admm", "polish-only"])
def test_pinned_cluttered_subset(gpu_available, admm):
    b = gen.with_pinned_velocity(gen.gen_cfg1(indices=range(400)))
    print(f"case: 400 cluttered edges, pinned start velocity, admm={admm}", flush=True)
    _, out = solve(b, None if admm else polish_only())
    r = compare(b, out["P"], out["cost"], out["status"], out["kkt"], label="pinned400")
    assert r["solved"] > 100


def test_pinned_mixed_degrees(gpu_available):
    b = gen.with_pinned_velocity(gen.gen_cfg2(indices=range(300)))
    print("case: 300 uneven segments, pinned start velocity", flush=True)
    _, out = solve(b)
    compare(b, out["P"], out["cost"], out["status"], out["kkt"], label="pinned-uneven")


def test_pinned_full_size(gpu_available):
    b = gen.with_pinned_velocity(gen.generate(1, 50_000))
    print("case: 50k cluttered edges, pinned start velocity", flush=True)
    _, out = solve(b, polish_only())
    st = out["status"]
    assert set(np.unique(st).tolist()) <= {qp.SOLVED, qp.INFEASIBLE}
    ok = st == qp.SOLVED
    assert np.all(out["kkt"][ok] <= KKT_TOL)
    v = start_velocity(b, out["P"])
    assert np.abs(v[ok] - b.x0[ok, 3:]).max() <= 1e-9
    idx = np.random.default_rng(31).choice(b.n, 200, replace=False)
    compare(b, out["P"], out["cost"], st, out["kkt"], idx=idx, label="pinned50k")


def test_start_speed_above_vmax(gpu_available):
    b = gen.with_pinned_velocity(gen.gen_cfg1(indices=range(64)))
    b.x0[:32, 3] = np.where(np.arange(32) % 2, 1.0, -1.0) * (b.vmax + 0.25)
    _, out = solve(b)
    assert np.all(out["status"][:32] == qp.INFEASIBLE) and np.all(np.isinf(out["cost"][:32]))
    compare(b, out["P"], out["cost"], out["status"], out["kkt"], idx=range(32, 64), label="pinned-rest")


def test_pinned_backward_matches_oracle(gpu_available):
    from paper_2411_13507_amd.api import SegmentBatchGPU
    sub = gen.gen_cfg1(indices=range(300))
    b = gen.with_pinned_velocity(gen.from_instances([sub.instance(i) for i in range(sub.n)]))
    gbar = gen.upstream_grads(4, b.n)
    gb = SegmentBatchGPU(b)
    d = gb.device
    res = gb.solve(torch.as_tensor(b.x0, device=d), torch.as_tensor(b.goal, device=d))
    g = gb.backward(torch.as_tensor(gbar.ravel(), device=d), torch.ones(b.n, dtype=torch.float64, device=d))
    torch.cuda.synchronize()
    st = res.status.cpu().numpy()
    gx0, ggoal, gbi = g.x0.cpu().numpy(), g.goal.cpu().numpy(), g.b_inst.cpu().numpy()

    def rel(a, c):
        return np.linalg.norm(a - c) / max(np.linalg.norm(c), 1e-8)
    n_checked = n_pin = 0
    worst = 0.0
    for i in range(b.n):
        if st[i] != qp.SOLVED:
            assert np.all(gx0[i] == 0)
            continue
        o = segment.solve(b.instance(i))
        if not segment.gradient_certified(o):
            continue
        ox0, ogoal, ob = segment.gradients(o, gbar[i]).combined(1.0)
        f0, f1 = gb.face_off[i], gb.face_off[i + 1]
        e = max(rel(gx0[i], ox0), rel(ggoal[i], ogoal), rel(gbi[f0:f1], ob) if np.linalg.norm(ob) > 1e-8 else 0.0)
        worst = max(worst, e)
        assert e <= GRAD_RTOL, (i, e, gx0[i], ox0)
        n_checked += 1
        n_pin += np.linalg.norm(ox0[3:]) > 1e-6
    print(f"pinned backward vs oracle: {n_checked} instances ({n_pin} with d/dv0 != 0), worst {worst:.2e}",
          flush=True)
    assert n_checked >= 40 and n_pin >= 20
    gb.close()
