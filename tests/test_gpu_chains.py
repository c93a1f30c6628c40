"""GPU path solver (segments joined with C0/C1/C2 continuity) against the FP64
oracle, through the C ABI."""
import multiprocessing as mp

import numpy as np
import pytest
import torch

from oracle import chain as ochain
from oracle import qp
from tests.parity_helpers import COST_ATOL, COST_RTOL, KKT_TOL, P_TOL
from workloads import gen

pytestmark = pytest.mark.gpu


def gpu_chains(b, opts=None):
    from paper_2411_13507_amd.api import ChainBatchGPU
    cb = ChainBatchGPU(b)
    x0 = torch.as_tensor(b.x0, device=cb.device)
    goal = torch.as_tensor(b.goal, device=cb.device)
    res = cb.solve(x0, goal, opts=opts)
    torch.cuda.synchronize()
    return cb, dict(P=res.P.cpu().numpy(), cost=res.cost.cpu().numpy(), status=res.status.cpu().numpy(),
                    kkt=res.kkt.cpu().numpy(), iters=res.iters.cpu().numpy())


def _orc(ch):
    r = ochain.solve(ch)
    return dict(status=r.status, cost=r.cost, P=r.P, s=r.s_star)


def compare_chains(b, out, idx, label):
    with mp.get_context("fork").Pool(8) as pool:
        orc = pool.map(_orc, [b.chain(i) for i in idx])
    p = b.degree
    mism, worst_c, worst_p, n_solved = [], 0.0, 0.0, 0
    for o, i in zip(orc, idx):
        st = int(out["status"][i])
        if o["status"] in (qp.SOLVED, qp.INFEASIBLE) and st != o["status"]:
            mism.append((int(i), o["status"], st, o["s"]))
            continue
        if o["status"] == qp.SOLVED:
            n_solved += 1
            a, z = b.seg_off[i], b.seg_off[i + 1]
            Pg = out["P"][3 * (p + 1) * a:3 * (p + 1) * z].reshape(-1, p + 1, 3)
            ce = abs(out["cost"][i] - o["cost"])
            assert ce <= COST_RTOL * abs(o["cost"]) + COST_ATOL, (label, i, out["cost"][i], o["cost"])
            pe = np.abs(Pg - o["P"]).max() / (1 + np.abs(o["P"]).max())
            assert pe <= P_TOL, (label, i, pe)
            assert out["kkt"][i] <= KKT_TOL
            worst_c = max(worst_c, ce / (abs(o["cost"]) + 1e-3))
            worst_p = max(worst_p, pe)
    print(f"{label}: {len(idx)} paths, {n_solved} solved, status mismatches {mism[:5]}, "
          f"worst cost err {worst_c:.2e}, worst P err {worst_p:.2e}", flush=True)
    assert not mism


def _opts(admm):
    if admm is None:
        return None
    from paper_2411_13507_amd import _lib
    o = _lib.default_opts()
    o.admm_iters = admm
    return o


@pytest.mark.parametrize("admm", [None, 0], ids=["default", "polish-only"])
def test_chain_subset(gpu_available, admm):
    b = gen.gen_cfg3(indices=range(48))
    print(f"case: 48 paths of 4-12 segments, admm_iters {admm}", flush=True)
    _, out = gpu_chains(b, _opts(admm))
    compare_chains(b, out, list(range(b.n)), "paths48")


@pytest.mark.parametrize("admm", [None, 0], ids=["default", "polish-only"])
def test_chain_full_size_sampled(gpu_available, admm):
    """Every path of the 8,192-path batch ends SOLVED (KKT residual within
    tolerance) or INFEASIBLE with a verified certificate.  Compared with the
    oracle: every path the GPU calls infeasible (the oracle must agree where
    it certifies, and never solve it), the 24 paths that took the most polish
    steps, and 48 random paths."""
    b = gen.gen_cfg3(8192)
    print(f"case: 8192 paths, admm_iters {admm}", flush=True)
    _, out = gpu_chains(b, _opts(admm))
    st = out["status"]
    print(f"paths8192: {np.bincount(st, minlength=4).tolist()} (solved, infeasible, -, no verified answer)", flush=True)
    assert set(np.unique(st).tolist()) <= {qp.SOLVED, qp.INFEASIBLE}, np.bincount(st)
    assert np.all(out["kkt"][st == qp.SOLVED] <= KKT_TOL)
    hard = np.argsort(-out["iters"][:, 1], kind="stable")[:24]
    rnd = np.random.default_rng(77).choice(b.n, 48, replace=False)
    idx = np.unique(np.concatenate([np.where(st == qp.INFEASIBLE)[0], hard, rnd]))
    compare_chains(b, out, [int(i) for i in idx], "paths8192-infeasible+hardest+sampled")


def test_single_segment_path_matches_segment_solver(gpu_available):
    """A one-segment path is the segment problem: both GPU solvers must agree."""
    from paper_2411_13507_amd.api import SegmentBatchGPU
    seg = gen.gen_cfg1(indices=range(40))
    ch = gen.ChainBatch(
        name="one-segment", degree=7, T=1.0, vmax=seg.vmax, amax=seg.amax,
        seg_off=np.arange(seg.n + 1, dtype=np.int64), poly_off=seg.poly_off, A_face=seg.A_face,
        b_face=seg.b_face, poly_idx=seg.poly_idx, reach_off=seg.reach_off, H_off=seg.H_off, H=seg.H,
        h0=seg.h0, G=seg.G, x0=seg.x0, goal=seg.goal)
    _, oc = gpu_chains(ch)
    gb = SegmentBatchGPU(seg)
    r = gb.solve(torch.as_tensor(seg.x0, device=gb.device), torch.as_tensor(seg.goal, device=gb.device))
    torch.cuda.synchronize()
    st = r.status.cpu().numpy()
    assert np.array_equal(st, oc["status"])
    ok = st == 0
    P1 = r.P.cpu().numpy().reshape(seg.n, -1)[ok]
    P2 = oc["P"].reshape(seg.n, -1)[ok]
    assert np.abs(P1 - P2).max() <= 1e-9 * (1 + np.abs(P1).max())
    assert np.allclose(r.cost.cpu().numpy()[ok], oc["cost"][ok], rtol=1e-9, atol=1e-11)


def test_chain_admm_iteration_counts(gpu_available):
    """Polish alone and a long warm start reach the same optima."""
    from paper_2411_13507_amd import _lib
    b = gen.gen_cfg3(indices=range(24))
    outs = {}
    for k in (0, 10, 60):
        o = _lib.default_opts()
        o.admm_iters = k
        _, outs[k] = gpu_chains(b, o)
    for k in (0, 60):
        assert np.array_equal(outs[k]["status"], outs[10]["status"])
        ok = outs[10]["status"] == 0
        assert np.nanmax(np.abs(outs[k]["P"] - outs[10]["P"])) <= 1e-8
    print("mean polish steps by ADMM iterations", {k: float(v["iters"][:, 1].mean()) for k, v in outs.items()})
    compare_chains(b, outs[0], list(range(b.n)), "paths-polish-only")


def test_chain_graph_capture_replays(gpu_available):
    """Both launches of the path solve -- the reduced-cap pass and the
    full-cap pass that re-solves the paths marked for retry, reading the
    statuses the first wrote -- replay from one captured graph with the eager
    results, replay after replay."""
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import ChainBatchGPU
    b = gen.gen_cfg3(indices=range(256))
    print("case: 256 paths, graph capture of the polish-only solve", flush=True)
    cb = ChainBatchGPU(b)
    d = cb.device
    x0, goal = torch.as_tensor(b.x0, device=d), torch.as_tensor(b.goal, device=d)
    o = _lib.default_opts()
    o.admm_iters = 0
    ref = cb.solve(x0, goal, opts=o)
    torch.cuda.synchronize()
    want = [t.clone() for t in (ref.P, ref.cost, ref.status, ref.kkt)]
    assert int((want[2] == 0).sum()) > 0
    out = cb.solve(x0, goal, opts=o)
    side = torch.cuda.Stream(device=d)
    side.wait_stream(torch.cuda.current_stream(d))
    with torch.cuda.stream(side):
        cb.solve(x0, goal, opts=o, out=out)
    torch.cuda.current_stream(d).wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cb.solve(x0, goal, opts=o, out=out)
    for rep in range(3):
        out.P.fill_(7.0)
        out.status.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        for a, w in zip((out.P, out.cost, out.status, out.kkt), want):
            assert torch.equal(a, w) or torch.allclose(a, w, rtol=0.0, atol=0.0, equal_nan=True), rep
        cb.solve(x0, goal, opts=o)
        torch.cuda.synchronize()
