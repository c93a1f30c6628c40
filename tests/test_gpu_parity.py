"""GPU forward pass against the FP64 oracle, through the C ABI.

Workloads: the 64-segment box batch in full, seeded subsets of the
cluttered-environment batch (degree 7, 8-24 faces) and of the uneven batch
(degree 3-9, 6-40 faces, 16-128 reachable rows), the full 50,000-edge batch
in the benchmark's launch configuration (sampled against the oracle, the
rest by properties), and edge cases."""
import numpy as np
import pytest
import torch

from oracle import qp
from tests.parity_helpers import KKT_TOL, compare
from workloads import gen

pytestmark = pytest.mark.gpu

def gpu_solve(batch, opts=None, b_face=None, x0=None, goal=None):
    from paper_2411_13507_amd.api import SegmentBatchGPU
    gb = SegmentBatchGPU(batch)
    x0 = torch.as_tensor(batch.x0 if x0 is None else x0, device=gb.device).contiguous()
    goal = torch.as_tensor(batch.goal if goal is None else goal, device=gb.device).contiguous()
    bf = None if b_face is None else torch.as_tensor(b_face, device=gb.device).contiguous()
    res = gb.solve(x0, goal, b_face=bf, opts=opts)
    torch.cuda.synchronize()
    out = dict(P=res.P.cpu().numpy(), cost=res.cost.cpu().numpy(), status=res.status.cpu().numpy(),
               kkt=res.kkt.cpu().numpy(), iters=res.iters.cpu().numpy())
    return gb, out


def opts(**kw):
    from paper_2411_13507_amd import _lib
    o = _lib.default_opts()
    names = {f[0] for f in _lib.SolveOpts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise AttributeError(f"rbp_solve_opts has no field {k!r}")
        setattr(o, k, v)
    return o


def check(batch, out, idx=None, label=""):
    return compare(batch, out["P"], out["cost"], out["status"], out["kkt"], idx=idx, label=label)


def test_cfg0_full(gpu_available):
    b = gen.gen_cfg0(64)
    print("case: 64 box segments, degree 7", flush=True)
    _, out = gpu_solve(b)
    r = check(b, out, label="seg64")
    assert r["solved"] > 10 and r["certified"] == 64


def test_cfg1_subset(gpu_available):
    b = gen.gen_cfg1(indices=range(400))
    print("case: 400 cluttered edges", flush=True)
    _, out = gpu_solve(b)
    check(b, out, label="edges400")


def test_cfg2_subset_mixed_degrees(gpu_available):
    b = gen.gen_cfg2(indices=range(300))
    assert len(set(b.degree.tolist())) == 7
    print("case: 300 uneven segments", flush=True)
    _, out = gpu_solve(b)
    check(b, out, label="uneven300")


def test_cfg1_full_size_sampled(gpu_available):
    """The 50,000-edge batch as the benchmark launches it: 256 seeded
    samples against the oracle, every instance by properties."""
    b = gen.generate(1, 50_000)
    print("case: 50k cluttered edges", flush=True)
    _, out = gpu_solve(b)
    st = out["status"]
    assert set(np.unique(st).tolist()) <= {qp.SOLVED, qp.INFEASIBLE}
    assert np.all(out["kkt"][st == qp.SOLVED] <= KKT_TOL)
    assert np.all(np.isinf(out["cost"][st == qp.INFEASIBLE]))
    assert 0.2 <= np.mean(st == qp.INFEASIBLE) <= 0.42
    idx = np.sort(np.random.default_rng(2024).choice(b.n, 256, replace=False))
    check(b, out, idx=idx, label="edges50k-sampled")


@pytest.mark.parametrize("admm_iters", [0, 200])
def test_polish_alone_and_long_admm(gpu_available, admm_iters):
    b = gen.gen_cfg1(indices=range(200))
    _, out = gpu_solve(b, opts(admm_iters=admm_iters))
    check(b, out, label=f"admm{admm_iters}")


def test_admm_warm_start_reduces_polish_steps(gpu_available):
    """The FP32 iterations (with the matrix-core Gram) must propose a useful
    working set: more iterations, fewer FP64 polish steps."""
    b = gen.gen_cfg1(indices=range(400))
    steps = {}
    for k in (0, 10, 100):
        _, out = gpu_solve(b, opts(admm_iters=k))
        steps[k] = out["iters"][:, 1].mean()
    print("mean polish steps by ADMM iterations", steps, flush=True)
    assert steps[10] < steps[0] and steps[100] < steps[0]


def test_plain_fp64_launch_per_instance_matches(gpu_available):
    b = gen.gen_cfg0(64)
    _, fast = gpu_solve(b)
    _, plain = gpu_solve(b, opts(plain=1))
    assert np.array_equal(fast["status"], plain["status"])
    ok = fast["status"] == qp.SOLVED
    assert np.nanmax(np.abs(fast["P"] - plain["P"])) <= 1e-9
    assert np.allclose(fast["cost"][ok], plain["cost"][ok], rtol=1e-9, atol=1e-12)
    check(b, plain, label="plain")


def test_b_face_override(gpu_available):
    b = gen.gen_cfg1(indices=range(120))
    rng = np.random.default_rng(7)
    bf = b.b_face + rng.uniform(-0.05, 0.1, b.b_face.shape)
    _, out = gpu_solve(b, b_face=bf)
    moved = gen.SegmentBatch(**{**b.__dict__, "b_face": bf})
    check(moved, out, label="b_override")


def test_determinism_and_order_independence(gpu_available):
    b = gen.gen_cfg1(indices=range(300))
    _, o1 = gpu_solve(b)
    _, o2 = gpu_solve(b)
    for k in ("P", "cost", "status", "kkt", "iters"):
        assert np.array_equal(o1[k], o2[k], equal_nan=True), k
    perm = np.random.default_rng(3).permutation(b.n)
    bp = b.subset(perm)
    _, op = gpu_solve(bp)
    P1 = o1["P"].reshape(b.n, -1)[perm]
    assert np.array_equal(P1, op["P"].reshape(b.n, -1), equal_nan=True)
    assert np.array_equal(o1["status"][perm], op["status"])


def _line(p=7, seed=0):
    from tests.test_oracle_qp import line_instance
    d = line_instance(p=p, seed=seed)
    d["vmax"], d["amax"] = 10.0, 10.0
    return d


def test_empty_batch(gpu_available):
    b = gen.from_instances([])
    gb, out = gpu_solve(b)
    assert out["status"].size == 0


def test_edge_cases(gpu_available):
    insts, expect = [], []
    d = _line(7, 1); insts.append(d); expect.append(qp.SOLVED)                       # no active row
    d = _line(7, 2); d["goal"] = d["x0"][:3] + np.array([25.0, 0, 0]); insts.append(d)
    expect.append(qp.INFEASIBLE)                                                       # goal outside polytope
    d = _line(7, 3); d["goal"] = d["x0"][:3] + np.array([10.5, 0, 0]); insts.append(d)
    expect.append(qp.INFEASIBLE)                                                       # beyond vmax T
    d = _line(7, 4); d["x0"] = d["x0"].copy(); d["x0"][1] = np.nan; insts.append(d)
    expect.append(5)                                                                   # invalid input
    d = _line(7, 5); d["T"] = -1.0; insts.append(d); expect.append(5)
    d = _line(7, 6); d["H"] = np.zeros((0, 24)); d["h0"] = np.zeros(0); d["G"] = np.zeros((0, 6))
    insts.append(d); expect.append(qp.SOLVED)                                          # no reachable rows
    b = gen.from_instances(insts)
    _, out = gpu_solve(b)
    assert out["status"].tolist() == expect, out["status"]
    assert abs(out["cost"][0]) <= 1e-9
    k = np.arange(8)[:, None] / 7
    line = insts[0]["x0"][:3] + k * (insts[0]["goal"] - insts[0]["x0"][:3])
    assert np.abs(out["P"][:24].reshape(8, 3) - line).max() <= 1e-9
    assert np.isinf(out["cost"][1]) and np.isinf(out["cost"][2])
    assert np.all(np.isnan(out["P"][3 * 8 * 3:3 * 8 * 4]))
    check(b, out, idx=[0, 1, 2, 5], label="edge")


def test_maximum_sizes(gpu_available):
    """Degree 9, 64 faces, 128 reachable rows (the largest instance the
    library accepts), mixed with a degree-3 instance in one launch."""
    rng = np.random.default_rng(99)
    insts = []
    for p, nf, r in ((9, 64, 128), (3, 6, 16), (9, 64, 128), (5, 40, 1)):
        c = rng.uniform(3, 7, 3)
        A = rng.standard_normal((nf, 3)); A /= np.linalg.norm(A, axis=1, keepdims=True)
        A[:6] = np.concatenate([np.eye(3), -np.eye(3)])
        bb = A @ c + rng.uniform(1.0, 2.0, nf)
        H = rng.standard_normal((r, 3 * (p + 1))); H /= np.linalg.norm(H, axis=1, keepdims=True)
        G = rng.normal(0, 0.1, (r, 6)); G[:, :3] += H.reshape(r, p + 1, 3).sum(1)
        x0 = np.concatenate([c + rng.uniform(-0.3, 0.3, 3), rng.uniform(-1, 1, 3)])
        insts.append(dict(p=p, T=1.0, vmax=3.0, amax=5.0, A_face=A, b_face=bb, H=H,
                          h0=rng.uniform(1.5, 3.5, r), G=G, x0=x0, goal=c + rng.uniform(-0.5, 0.5, 3)))
    b = gen.from_instances(insts)
    _, out = gpu_solve(b)
    check(b, out, label="max-size")


@pytest.mark.parametrize("schedule", [0, 1])
def test_graph_capture_replays_match_eager(gpu_available, schedule):
    """solve + backward captured in one graph on torch's stream; every replay
    (with eager work and synchronisations in between) must equal the eager
    results bitwise, for the grouped launches (schedule 0) and the single
    launch over the whole batch (schedule 1)."""
    from paper_2411_13507_amd.api import SegmentBatchGPU
    b = gen.gen_cfg2(indices=range(160))
    gb = SegmentBatchGPU(b)
    so = opts(schedule=schedule) if schedule else None
    dev = gb.device
    x0 = torch.as_tensor(b.x0, device=dev)
    goal = torch.as_tensor(b.goal, device=dev)
    gP = torch.as_tensor(np.random.default_rng(5).standard_normal(3 * gb.points_total), device=dev)
    gC = torch.ones(b.n, dtype=torch.float64, device=dev)
    out = gb.alloc_outputs()
    gb.solve(x0, goal, out=out, opts=so)
    gr = gb.backward(gP, gC)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (out.P, out.cost, out.status, out.kkt, gr.x0, gr.goal, gr.b_inst)]
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        gb.solve(x0, goal, out=out, opts=so)
        gb.backward(gP, gC, out=gr)
    torch.cuda.current_stream(dev).wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gb.solve(x0, goal, out=out, opts=so)
        gb.backward(gP, gC, out=gr)
    for rep in range(4):
        for t in (out.P, out.cost, out.kkt, gr.x0, gr.goal, gr.b_inst):
            t.fill_(-7.0)
        graph.replay()
        torch.cuda.synchronize()
        got = (out.P, out.cost, out.status, out.kkt, gr.x0, gr.goal, gr.b_inst)
        for a, r in zip(got, ref):
            assert torch.equal(torch.nan_to_num(a, nan=1.5), torch.nan_to_num(r, nan=1.5)), rep
        # eager work between replays
        gb.solve(x0 + 0.0, goal, out=gb.alloc_outputs(), opts=so)
        torch.cuda.synchronize()


def test_autotune_picks_a_candidate_and_results_do_not_change(gpu_available, tmp_path, monkeypatch):
    from paper_2411_13507_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    b = gen.gen_cfg1(indices=range(600))
    o = autotune.tune(b, sample=600, reps=2)
    assert (o.admm_iters, round(o.rho, 6)) in {(k, round(r, 6)) for k, r in autotune.CANDIDATES}
    assert (o.schedule, o.launch_shape) in autotune.LAUNCHES
    assert autotune.cached(b) is not None
    _, tuned = gpu_solve(b, o)
    _, default = gpu_solve(b)
    assert np.array_equal(tuned["status"], default["status"])
    ok = default["status"] == 0
    assert np.nanmax(np.abs(tuned["P"] - default["P"])) <= 1e-9
    check(b, tuned, label="autotuned")


@pytest.mark.parametrize("schedule,shape", [(1, 0), (0, 1), (0, 2)], ids=["single-launch", "one-wave-per-simd",
                                                                       "two-instances-per-workgroup"])
def test_schedules_and_launch_shapes_match_the_default(gpu_available, schedule, shape):
    """The single launch over the whole batch and the other launch shapes of
    the grouped schedule compute every instance as the default launches do
    (same statuses, P* and costs to 1e-12, same polish step counts), the
    backward pass of each matches too, and a second call gives the same
    bits; a sample is checked against the oracle."""
    from paper_2411_13507_amd.api import SegmentBatchGPU
    b = gen.gen_cfg2(indices=range(1500))
    print(f"case: 1500 uneven segments, schedule {schedule}, launch shape {shape}", flush=True)
    o_def = opts(admm_iters=0)
    o_var = opts(admm_iters=0, schedule=schedule, launch_shape=shape)
    gb = SegmentBatchGPU(b)
    dev = gb.device
    x0, goal = torch.as_tensor(b.x0, device=dev), torch.as_tensor(b.goal, device=dev)
    gP = torch.as_tensor(np.random.default_rng(5).standard_normal(3 * gb.points_total), device=dev)
    gC = torch.ones(b.n, dtype=torch.float64, device=dev)
    outs = []
    for o in (o_def, o_var, o_var):
        r = gb.solve(x0, goal, opts=o)
        g = gb.backward(gP, gC)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in (("P", r.P), ("cost", r.cost), ("status", r.status),
                                                      ("kkt", r.kkt), ("iters", r.iters), ("gx0", g.x0),
                                                      ("gb", g.b_inst))})
    d, v, v2 = outs
    assert np.array_equal(d["status"], v["status"])
    assert np.array_equal(d["iters"], v["iters"])
    for k in ("P", "cost", "gx0", "gb"):
        a, c = np.nan_to_num(d[k], nan=0.0, posinf=0.0), np.nan_to_num(v[k], nan=0.0, posinf=0.0)
        assert np.abs(a - c).max() <= 1e-12 * (1.0 + np.abs(a).max()), k
    for k in v:
        assert np.array_equal(v[k], v2[k], equal_nan=True), k
    check(b, v, idx=list(range(0, b.n, 5)), label=f"uneven-schedule{schedule}-shape{shape}")
