"""Throughput of the batched segment-QP path on one MI355X.

A step is one pass of the whole path over the 50,000-edge cluttered
environment batch (degree-7 segments, 8-24 faces, 32 reachable rows, about
30% infeasible): the forward solve (rbp_solve_batch: an optional FP32 ADMM
stage, then the FP64 active-set polish that decides every result) followed
by the implicit-KKT backward (rbp_backward), inputs resident in HBM.  The
solve options are the autotuner's pick for the batch; the line also reports
the other precision form (FP32 ADMM + FP64 polish when the pick skips the
ADMM), each with its own dtype.  The value counts instances that end SOLVED
with a scaled KKT residual <= 1e-6 or INFEASIBLE with a verified
certificate.  Printed as one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP64, and FP32 without packing)
PEAK_HBM_GBS = 8000.0
KKT_OK = 1e-6


def instance_sizes(b):
    p = b.degree.astype(np.int64)
    nf = np.diff(b.poly_off.astype(np.int64))[b.poly_idx]
    r = np.diff(b.reach_off)
    if getattr(b, "reach_idx", None) is not None:
        r = r[b.reach_idx]
    return p, nf, r


def algorithmic_flops(b, iters):
    """Flops per instance of the forward kernel, from the instance sizes and
    the measured iteration counts (ADMM iterations, polish steps).  The ADMM
    set-up (reachable-row Gram, K and its inverse) is counted only for
    instances that ran ADMM iterations: the polish-only kernel never forms
    them."""
    p, nf, r = instance_sizes(b)
    n = 3 * (p - 1)
    F = (p - 1) * nf
    m = F + 6 * p - 3 + r
    nnz_diff = 3 * (2 * p - 2) + 3 * (3 * (p - 1) - 2)
    nnz = 3 * F + nnz_diff + r * n                         # free columns
    nnz_full = 3 * F + 6 * p + 9 * (p - 1) + r * 3 * (p + 1)
    admm_it = 4 * nnz + 2 * n * n + 10 * m
    setup = 2 * r * n * n + 2 * n ** 3 + r * 3 * (p - 1) * p + 2 * r * 3 * (p + 1) + 2 * n * n
    polish_step = 2 * nnz_full + 4 * n * n + n * (p - 1) + (n * n) // 4
    final = 2 * nnz_full + n * n + 2 * (3 * (p + 1)) ** 2
    K = iters[:, 0].astype(np.int64)
    S = iters[:, 1].astype(np.int64)
    return np.where(K > 0, setup, 0) + K * admm_it + S * polish_step + final


def algorithmic_bytes(b, q_mean=3, store=True):
    """HBM bytes per instance of the forward kernel: problem data read once,
    outputs written once and, when kept for the backward pass, the final
    working set (q_mean rows: ids, sides, multipliers), its factor (q_mean
    rows of Q1 over the 3(p-1) free variables and the upper triangle of R) and
    the six multipliers of the pinned start and goal coordinates."""
    p, nf, r = instance_sizes(b)
    if getattr(b, "reach_idx", None) is None:
        reads = 8 * r * 3 * (p + 1) + 48 * r + 8 * r + 72 + 8 + 44 + 32 * nf
    else:                                    # shared blocks: read once per launch, not per instance
        reads = 72 + 8 + 44 + 32 * nf + 4 + (8 * b.H.size + 56 * b.h0.size) / max(b.n, 1)
    n = 3 * (p - 1)
    kept = 16 * q_mean + 8 * (q_mean * n + q_mean * (q_mean + 1) / 2) + 48
    writes = 24 * (p + 1) + 16 + 4 + 8 + 4 + (kept if store else 0)
    return reads + writes


def roofline_record(flops, nbytes, t_launch):
    """Bound of a launch from its algorithmic work: the resource whose time
    at peak is larger (t_HBM = bytes / 8 TB/s, t_ALU = flops / 78.6 TFLOP/s)
    is the binding one, and ``frac`` is achieved / peak for that resource."""
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    t_alu = flops / (PEAK_VALU_TFLOPS * 1e12)
    if t_hbm >= t_alu:
        ach, peak, unit, bound = nbytes / t_launch / 1e9, PEAK_HBM_GBS, "GB/s", "hbm"
    else:
        ach, peak, unit, bound = flops / t_launch / 1e12, PEAK_VALU_TFLOPS, "TFLOP/s", "alu"
    return {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
            "t_hbm_us": t_hbm * 1e6, "t_alu_us": t_alu * 1e6, "bytes_per_launch": nbytes,
            "flops_per_launch": flops,
            "alu_frac": flops / t_launch / 1e12 / PEAK_VALU_TFLOPS,
            "hbm_frac": nbytes / t_launch / 1e9 / PEAK_HBM_GBS}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rbp_kernels.hip", "rbp_segment.hpp", "rbp_api.cpp", "rbp_internal.hpp", "rbp_consts.hpp", "rbp_wave.hpp"):
        with open(os.path.join(ROOT, "paper_2411_13507_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_inst):
    """HBM bytes per solve launch measured by rocprofv3 (FETCH_SIZE +
    WRITE_SIZE, scaled by the copy-kernel calibration), if taken on the
    current kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", "solve_edges50k_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash() or rec.get("instances") != n_inst:
        return None
    return float(rec["bytes_per_launch"])


def _oracle_fwd_bwd(args):
    from oracle import segment
    inst, gbar = args
    r = segment.solve(inst)
    g = None
    if segment.is_solved(r):
        g = segment.gradients(r, gbar).combined(1.0)
    return r.status, r.cost, r.P, g, segment.gradient_certified(r) if g is not None else False


def cpu_baseline(b, gbar, n_sample=2000):
    """The FP64 oracle (phase-1 LP + active set + gradients) on the first
    ``n_sample`` instances, over a process pool on the host cores.  Returns
    the baseline record and the oracle's results (for the error figures)."""
    import multiprocessing as mp
    cores = min(16, os.cpu_count() or 1)
    insts = [(b.instance(i), gbar[i]) for i in range(n_sample)]
    t = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_fwd_bwd, insts, chunksize=16)
    dt = time.perf_counter() - t
    return ({"value": n_sample / dt, "unit": "solves/s", "cores": cores, "kind": "oracle",
             "sample": f"first {n_sample} of the 50,000 edges, forward + gradients, {dt:.1f} s wall"}, res)


def errors_vs_oracle(b, orc, P, cost, status, gx0, ggoal, gb_inst):
    """Per-result error of the GPU outputs against the FP64 oracle on the
    instances the oracle ran (the first len(orc) of the batch): status
    mismatches on certified instances, max relative cost error, max P* error
    (|dP|_inf / (1 + |P|_inf)) and max gradient error (|dg|_2 / max(|g|_2,
    1e-8), over instances whose gradient is well defined)."""
    from oracle import qp
    pt_off = np.concatenate([[0], np.cumsum(b.degree.astype(np.int64) + 1)])
    nf = np.diff(b.poly_off.astype(np.int64))[b.poly_idx]
    f_off = np.concatenate([[0], np.cumsum(nf)])
    mism = cmp_ = 0
    ce = pe = ge = 0.0
    n_grad = 0
    for i, (ost, ocost, oP, og, gcert) in enumerate(orc):
        if ost in (qp.SOLVED, qp.INFEASIBLE):
            mism += int(status[i] != ost)
        if ost != qp.SOLVED or status[i] != qp.SOLVED:
            continue
        cmp_ += 1
        ce = max(ce, abs(cost[i] - ocost) / (abs(ocost) + 1e-3))
        Pg = P[3 * pt_off[i]:3 * pt_off[i + 1]].reshape(-1, 3)
        pe = max(pe, float(np.abs(Pg - oP).max() / (1.0 + np.abs(oP).max())))
        if gcert:
            n_grad += 1
            for mine, ref in ((gx0[i], og[0]), (ggoal[i], og[1]), (gb_inst[f_off[i]:f_off[i + 1]], og[2])):
                ge = max(ge, float(np.linalg.norm(mine - ref) / max(np.linalg.norm(ref), 1e-8)))
    return {"instances": len(orc), "status_mismatches_certified": mism, "solved_compared": cmp_,
            "max_cost_rel_err": ce, "max_P_err": pe, "gradients_compared": n_grad, "max_grad_rel_err": ge,
            "tolerances": {"cost": "1e-6 rel + 1e-9", "P": 1e-6, "grad": 1e-4}}


def time_launches(fn, reps, stream):
    import torch
    fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs])) / 1e3


def mpc_flops_per_iteration(N, m):
    """Algorithmic FP64 flops of one interior-point iteration of the MPC
    kernel (mr = m + 4 unit rows per step, RT = N mr rows): per step the
    barrier Hessian (81 entries x mr rows x 3), the Riccati update (~1,000),
    two gradient builds (2 x 9 x mr x 2) and Riccati solves (2 x 150), the
    costate gradient (18 (15 + mr)) and scan (40); per row the residual,
    the two direction recoveries, step lengths and the update (~93)."""
    mr = m + 4
    return N * (243 * mr + 1000 + 36 * mr + 300 + 18 * (15 + mr) + 40) + N * mr * 93


def _variant(sb, main_opts, reps, stream):
    """Forward + backward and forward-only times of a variant of the
    50,000-edge batch."""
    import torch
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import SegmentBatchGPU
    dev = torch.device("cuda", 0)
    sg = SegmentBatchGPU(sb, device="cuda:0")
    sx0, sgoal = torch.as_tensor(sb.x0, device=dev), torch.as_tensor(sb.goal, device=dev)
    sres = sg.alloc_outputs()
    sgP = torch.as_tensor(np.random.default_rng(5).standard_normal(3 * sg.points_total), device=dev)
    sgC = torch.ones(sb.n, dtype=torch.float64, device=dev)
    holder = {}

    def fb():
        sg.solve(sx0, sgoal, opts=main_opts, out=sres)
        holder["g"] = sg.backward(sgP, sgC, out=holder.get("g"))
    t = time_launches(fb, reps, stream)
    fo = _lib.SolveOpts.from_buffer_copy(main_opts)
    fo.store_for_backward = 0
    t_f = time_launches(lambda: sg.solve(sx0, sgoal, opts=fo, out=sres), reps, stream)
    st = sres.status.cpu().numpy()
    kk = sres.kkt.cpu().numpy()
    ok = int(((st == 0) & (kk <= KKT_OK)).sum() + (st == 1).sum())
    rec = {"fwd_bwd_ms": t * 1e3, "solves_per_s": ok / t, "fwd_ms": t_f * 1e3, "instances": sb.n,
           "algorithmic_bytes_per_instance": float(algorithmic_bytes(sb).mean()),
           "status_counts": np.bincount(st, minlength=6).tolist()}
    if sb.reach_idx is not None:
        rec["reach_blocks"] = int(len(sb.reach_off) - 1)
    sg.close()
    return rec


def extra_workloads(reps=3, admm_iters=-1, edges=None, main_opts=None):
    """Throughput of the other workloads: the 50,000 edges with one shared
    reachable block and with a pinned start velocity, the uneven batch (200,000 segments, degree 3-9, 6-40
    faces, 16-128 reachable rows; autotuned options), the graph cut, graph
    building and adjacent hyperplanes, the path batch (8,192 paths of 4-12
    joined degree-7 segments) and the MPC refinement batch (4,096 horizons of
    50 steps)."""
    import torch
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import ChainBatchGPU, SegmentBatchGPU
    from workloads import gen
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream(dev)
    out = {}
    if edges is not None:
        # the same 50,000 edges with one reachable block shared by all, and
        # with the start velocity pinned (fwd + bwd with the headline options)
        out["edges50k_p7_shared_reach"] = _variant(gen.with_shared_reach(edges), main_opts, reps, stream)
        out["edges50k_p7_pinned_v0"] = _variant(gen.with_pinned_velocity(edges), main_opts, reps, stream)
    uneven_workload(out, reps, stream, admm_iters)
    # graph cut (Alg. 2 + Cut-QP): 50,000 edges x 200 box obstacles, codes and
    # per-edge collision counts (the cut graph)
    from paper_2411_13507_amd.api import CutGPU
    cb_ = gen.gen_cut()
    cg = CutGPU(cb_, cb_.n_edges, device="cuda:0")
    Pc = torch.as_tensor(cb_.P, device=dev)
    cres = cg.alloc()
    t = time_launches(lambda: cg.run(Pc, out=cres, with_step=False, with_dist=False), reps, stream)
    n_qp = cg.qp_count()
    cg.run(Pc, out=cres)
    steps = np.bincount(cres.step.cpu().numpy().ravel(), minlength=4)[1:].tolist()
    n_pairs = cb_.n_edges * cb_.n_obstacles
    out["cut50k_o200"] = {"ms": t * 1e3, "pairs_per_s": n_pairs / t, "edges": cb_.n_edges,
                          "obstacles": cb_.n_obstacles, "pairs_by_step": steps, "qp_pairs": n_qp,
                          "edges_cut": int((cres.n_collide.cpu().numpy() > 0).sum())}
    cg.close()
    del cres, Pc
    # the same edges against 200 boxes and 100 convex polytopes (8-16 faces):
    # codes and per-edge counts (as above), and separately with the step and
    # the Cut-QP values of the undecided pairs
    cbp = gen.gen_cut(n_poly=100)
    cgp = CutGPU(cbp, cbp.n_edges, device="cuda:0")
    Pcp = torch.as_tensor(cbp.P, device=dev)
    cresp = cgp.alloc()
    t = time_launches(lambda: cgp.run(Pcp, out=cresp, with_step=False, with_dist=False), reps, stream)
    t_val = time_launches(lambda: cgp.run(Pcp, out=cresp), reps, stream)
    cgp.run(Pcp, out=cresp)
    n_qp = cgp.qp_count()
    stp = cresp.step.cpu().numpy()
    n_pairs = cbp.n_edges * cbp.n_obstacles
    out["cut50k_o200_p100"] = {"ms": t * 1e3, "pairs_per_s": n_pairs / t, "ms_with_values": t_val * 1e3,
                               "edges": cbp.n_edges,
                               "boxes": cbp.n_boxes, "polytopes": cbp.n_polytopes,
                               "polytope_pairs_by_step": np.bincount(stp[cbp.n_boxes:].ravel(), minlength=4)[1:].tolist(),
                               "qp_pairs": n_qp, "edges_cut": int((cresp.n_collide.cpu().numpy() > 0).sum())}
    cgp.close()
    del cresp, Pcp
    # graph building (F1 v_i + F2 v_j <= G over all 25M ordered pairs of 5,000
    # nodes) in Z-order and in a random numbering (no tile skipping), and the
    # adjacent hyperplanes of the nodes against 200 boxes
    from paper_2411_13507_amd.api import GraphGPU, adjacent_hyperplanes
    gb_ = gen.gen_graph()
    gg = GraphGPU(gb_, gb_.V.shape[0], device="cuda:0")
    Vz = torch.as_tensor(gb_.V, device=dev)
    Vr = torch.as_tensor(gb_.V[np.random.default_rng(5).permutation(len(gb_.V))], device=dev)
    adj, deg = gg.run(Vz)
    t_z = time_launches(lambda: gg.run(Vz, adj, deg), reps, stream)
    n_edges = int(deg.sum().item())
    t_r = time_launches(lambda: gg.run(Vr, adj, deg), reps, stream)
    lo_, hi_ = torch.as_tensor(gb_.box_lo, device=dev), torch.as_tensor(gb_.box_hi, device=dev)
    t_h = time_launches(lambda: adjacent_hyperplanes(Vz, lo_, hi_), reps, stream)
    n_pairs = gb_.V.shape[0] ** 2
    out["graph5000_m64"] = {"ms_zorder": t_z * 1e3, "ms_random_order": t_r * 1e3, "edges": n_edges,
                            "pairs_per_s_zorder": n_pairs / t_z, "rows": int(gb_.F1.shape[0])}
    out["adjacent_hyperplanes_5000x200"] = {"ms": t_h * 1e3, "nodes": int(gb_.V.shape[0]),
                                            "obstacles": int(gb_.box_lo.shape[0])}
    gg.close()
    chains_workload(out, reps, stream)
    mpc_workload(out, reps, stream)
    return out


def uneven_workload(out, reps, stream, admm_iters=-1):
    """The uneven batch: 200,000 segments of degree 3-9, 6-40 faces, 16-128
    reachable rows, forward, with autotuned options (admm_iters < 0) captured
    in one HIP graph."""
    import torch
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import SegmentBatchGPU
    from workloads import gen
    dev = torch.device("cuda", 0)
    b = gen.generate(2, 200_000)
    gb = SegmentBatchGPU(b, device="cuda:0")
    x0, goal = torch.as_tensor(b.x0, device=dev), torch.as_tensor(b.goal, device=dev)
    res = gb.alloc_outputs()
    from paper_2411_13507_amd import autotune
    tuning = None
    if admm_iters >= 0:
        uo = _lib.default_opts()
        uo.admm_iters = admm_iters
    else:
        uo = autotune.tune(b, sample=b.n, reps=2, use_cache=False)
        tuning = autotune.tune.last
    uo.store_for_backward = 0
    # the tuned solve (every launch of its schedule) captured in one HIP graph
    gb.solve(x0, goal, opts=uo, out=res)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        gb.solve(x0, goal, opts=uo, out=res)
    stream.wait_stream(side)
    ugraph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(ugraph):
        gb.solve(x0, goal, opts=uo, out=res)
    t = time_launches(ugraph.replay, reps, stream)
    st = res.status.cpu().numpy()
    kk = res.kkt.cpu().numpy()
    ok = int(((st == 0) & (kk <= KKT_OK)).sum() + (st == 1).sum())
    out["uneven200k_p3to9"] = {"fwd_ms": t * 1e3, "solves_per_s": ok / t, "instances": b.n, "launch": "hipgraph",
                               "admm_iters": int(uo.admm_iters), "rho": round(float(uo.rho), 6),
                               "schedule": int(uo.schedule), "launch_shape": int(uo.launch_shape),
                               "status_counts": np.bincount(st, minlength=6).tolist(),
                               "tuning_ms": None if tuning is None else {"admm/rho": tuning["ms"],
                                                                         "launch": tuning["ms_launch"]}}
    del ugraph
    gb.close()
    del b, gb, res


def chains_workload(out, reps, stream):
    """8,192 paths of 4-12 joined degree-7 segments, forward (polish only)."""
    import torch
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import ChainBatchGPU
    from workloads import gen
    dev = torch.device("cuda", 0)
    c = gen.generate_chains(8192)
    cb = ChainBatchGPU(c, device="cuda:0")
    x0, goal = torch.as_tensor(c.x0, device=dev), torch.as_tensor(c.goal, device=dev)
    holder = {}
    # polish only: the dual active-set method started cold reaches the same
    # optima as after an ADMM warm start, in 2.5x less time on paths
    co = _lib.default_opts()
    co.admm_iters = 0
    t = time_launches(lambda: holder.__setitem__("r", cb.solve(x0, goal, opts=co, out=holder.get("r"))),
                      reps, stream)
    r = holder["r"]
    st = r.status.cpu().numpy()
    kk = r.kkt.cpu().numpy()
    ok = int(((st == 0) & (kk <= KKT_OK)).sum() + (st == 1).sum())
    nseg = int(c.seg_off[-1])
    out["chains8k_p7"] = {"fwd_ms": t * 1e3, "paths_per_s": ok / t, "paths": c.n, "segments": nseg,
                          "segment_solves_per_s": ok / t * nseg / c.n,
                          "status_counts": np.bincount(st, minlength=6).tolist(), "admm_iters": 0,
                          "polish_steps_mean": float(r.iters.cpu().numpy()[:, 1].mean())}
    cb.close()


def mpc_workload(out, reps, stream):
    """4,096 MPC refinements of 50 steps (eq. MPC)."""
    import torch
    from workloads import gen
    dev = torch.device("cuda", 0)
    # MPC refinement (eq. MPC): 4,096 independent 50-step horizons, one
    # separating plane per step, 16 reachable rows per step
    from paper_2411_13507_amd.api import MpcGPU
    mb = gen.gen_mpc(4096)
    mg = MpcGPU(mb, mb.n, device="cuda:0")
    mx0, mref, mpl = (torch.as_tensor(a, device=dev) for a in (mb.x0, mb.ref, mb.planes))
    mres = mg.alloc()
    t = time_launches(lambda: mg.solve(mx0, mref, mpl, out=mres), reps, stream)
    st = mres.status.cpu().numpy()
    its = mres.iters.cpu().numpy()
    ok = int((st == 0).sum())
    flops = float(mpc_flops_per_iteration(mb.N, int(mb.G.size)) * (its.astype(np.float64) + 1.0).sum())
    out["mpc4096_n50"] = {"ms": t * 1e3, "solves_per_s": ok / t, "instances": mb.n, "horizon": mb.N,
                          "reach_rows": int(mb.G.size), "status_counts": np.bincount(st, minlength=6).tolist(),
                          "ipm_iters_mean": float(its.mean()), "ipm_iters_max": int(its.max()),
                          "alu_tflops": flops / t / 1e12, "alu_frac": flops / t / 1e12 / PEAK_VALU_TFLOPS}
    mg.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=50_000)
    ap.add_argument("--admm-iters", type=int, default=-1,
                    help="ADMM warm-start iterations; -1 (default): options picked by the autotuner")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--workload", choices=["uneven", "chains", "mpc"], default=None,
                    help="only time this one workload of the extras and print its record (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 8, "copy_bytes_written": y.numel() * 8, "launches": 3}))
        return
    if args.workload is not None and args.gpus == 1:
        import torch
        dev = torch.device("cuda", 0)
        torch.cuda.set_device(dev)
        rec = {}
        st = torch.cuda.current_stream(dev)
        if args.workload == "uneven":
            uneven_workload(rec, max(args.steps, 1), st, args.admm_iters)
        else:
            {"chains": chains_workload, "mpc": mpc_workload}[args.workload](rec, max(args.steps, 1), st)
        print(json.dumps(rec))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); instances are independent, "
              "so a multi-GPU run would shard the batch with no communication.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2411_13507_amd import _lib
    from paper_2411_13507_amd.api import SegmentBatchGPU
    from workloads import gen

    b = gen.generate(1, args.n)
    gbar = gen.upstream_grads(4, b.n) if b.n <= 50_000 else np.random.default_rng(4).standard_normal((b.n, 24))
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    gb = SegmentBatchGPU(b, device="cuda:0")
    x0 = torch.as_tensor(b.x0, device=dev)
    goal = torch.as_tensor(b.goal, device=dev)
    gP = torch.as_tensor(gbar.ravel(), device=dev)
    gC = torch.ones(b.n, dtype=torch.float64, device=dev)
    if args.admm_iters >= 0:
        opts = _lib.default_opts()
        opts.admm_iters = args.admm_iters
        tuned = None
    else:
        # fastest options for this batch signature, timed on the whole batch
        # (every candidate reaches the same optima; see autotune.py)
        from paper_2411_13507_amd import autotune
        opts = autotune.tune(b, sample=b.n, reps=3, use_cache=False)
        tuned = {"admm_iters": int(opts.admm_iters), "rho": round(float(opts.rho), 6),
                 "schedule": int(opts.schedule), "launch_shape": int(opts.launch_shape),
                 "launch_ms": autotune.tune.last["ms_launch"]}
    out = gb.alloc_outputs()
    grads = None

    def step():
        nonlocal grads
        gb.solve(x0, goal, opts=opts, out=out)
        grads = gb.backward(gP, gC, out=grads)

    step()                                   # allocates the gradient buffers
    torch.cuda.synchronize()
    # capture one step (per-degree solve launches, state copies, backward) in a
    # HIP graph on torch's stream; replay it as the timed step
    launch = "hipgraph"
    run = step
    try:
        cur = torch.cuda.current_stream(dev)
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            step()
        cur.wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        run = graph.replay
    except Exception as exc:                 # capture refused: time the eager launches
        launch = f"eager (capture failed: {type(exc).__name__})"
        run = step
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    st = out.status.cpu().numpy()
    kkt = out.kkt.cpu().numpy()
    iters = out.iters.cpu().numpy()
    n_ok = int(((st == 0) & (kkt <= KKT_OK)).sum())
    n_inf = int((st == 1).sum())
    counted = n_ok + n_inf
    value = counted / dt

    # forward kernel alone, HIP events on the launch stream
    fopts = _lib.SolveOpts.from_buffer_copy(opts)
    fopts.store_for_backward = 0
    stream = torch.cuda.current_stream(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for _ in range(2):
        gb.solve(x0, goal, opts=fopts, out=out)
    for e0, e1 in evs:
        e0.record(stream)
        gb.solve(x0, goal, opts=fopts, out=out)
        e1.record(stream)
    torch.cuda.synchronize()
    t_solve = float(np.mean([e0.elapsed_time(e1) for e0, e1 in evs])) / 1e3
    # backward kernel alone
    gb.solve(x0, goal, opts=opts, out=out)
    bevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in bevs:
        e0.record(stream)
        gb.backward(gP, gC, out=grads)
        e1.record(stream)
    torch.cuda.synchronize()
    t_bwd = float(np.mean([e0.elapsed_time(e1) for e0, e1 in bevs])) / 1e3

    # roofline of the timed forward launch (store_for_backward off): only
    # the work that launch executes is counted
    fw_iters = out.iters.cpu().numpy()
    flops = float(algorithmic_flops(b, fw_iters).sum())
    nbytes = float(algorithmic_bytes(b, store=False).sum())
    roof = roofline_record(flops, nbytes, t_solve)
    roof["traffic"] = traffic_from_profile(b.n)
    admm_on = int(opts.admm_iters) > 0
    if int(opts.schedule) == 1:
        kernel_name = f"solve_kernel_all<{'true' if admm_on else 'false'}>"
    elif int(opts.launch_shape) != 0:
        wpg, wpe = {1: (1, 1), 2: (2, 2)}[int(opts.launch_shape)]
        kernel_name = f"solve_kernel_shape<7, {'true' if admm_on else 'false'}, {wpg}, {wpe}>"
    else:
        kernel_name = f"solve_kernel<float, 7, {'true' if admm_on else 'false'}>"
    dtype = "fp32+fp64" if admm_on else "fp64"
    roof["kernel"] = kernel_name
    roof["launch_ms"] = t_solve * 1e3
    # restore the headline forward + backward outputs for the error figures
    gb.solve(x0, goal, opts=opts, out=out)
    grads = gb.backward(gP, gC, out=grads)
    torch.cuda.synchronize()

    # the other precision form on the same batch: FP32 ADMM (MFMA Gram of the
    # reachable rows, K^-1 in registers) + FP64 polish when the tuned options
    # skip the ADMM, the polish alone otherwise
    alt_opts = _lib.default_opts()
    if admm_on:
        alt_opts.admm_iters = 0
    else:
        alt_opts.admm_iters = 10
    alt_opts.store_for_backward = 1
    alt_out = gb.alloc_outputs()
    alt_g = {}

    def alt_step():
        gb.solve(x0, goal, opts=alt_opts, out=alt_out)
        alt_g["g"] = gb.backward(gP, gC, out=alt_g.get("g"))
    t_alt = time_launches(alt_step, max(3, args.steps // 4), torch.cuda.current_stream(dev))
    alt_f = _lib.SolveOpts.from_buffer_copy(alt_opts)
    alt_f.store_for_backward = 0
    t_alt_f = time_launches(lambda: gb.solve(x0, goal, opts=alt_f, out=alt_out), max(3, args.steps // 4),
                            torch.cuda.current_stream(dev))
    a_st = alt_out.status.cpu().numpy()
    a_kk = alt_out.kkt.cpu().numpy()
    a_it = alt_out.iters.cpu().numpy()
    a_ok = int(((a_st == 0) & (a_kk <= KKT_OK)).sum() + (a_st == 1).sum())
    a_roof = roofline_record(float(algorithmic_flops(b, a_it).sum()), nbytes, t_alt_f)
    alt_rec = {"dtype": "fp64" if admm_on else "fp32+fp64", "admm_iters": int(alt_opts.admm_iters),
               "rho": round(float(alt_opts.rho), 6),
               "kernel": f"solve_kernel<float, 7, {'false' if admm_on else 'true'}>",
               "fwd_bwd_ms": t_alt * 1e3, "fwd_ms": t_alt_f * 1e3, "solves_per_s": a_ok / t_alt,
               "fwd_solves_per_s": a_ok / t_alt_f, "status_counts": np.bincount(a_st, minlength=6).tolist(),
               "polish_steps_mean": float(a_it[:, 1].mean()),
               "roofline": {k: a_roof[k] for k in ("bound", "achieved", "unit", "frac", "alu_frac", "hbm_frac")}}
    # gradients of the alternative form are needed for its error figures
    gb.solve(x0, goal, opts=alt_opts, out=alt_out)
    alt_grads = gb.backward(gP, gC, out=alt_g.get("g"))
    torch.cuda.synchronize()
    alt_np = (alt_out.P.cpu().numpy(), alt_out.cost.cpu().numpy(), alt_out.status.cpu().numpy(),
              alt_grads.x0.cpu().numpy(), alt_grads.goal.cpu().numpy(), alt_grads.b_inst.cpu().numpy())
    main_np = (out.P.cpu().numpy(), out.cost.cpu().numpy(), out.status.cpu().numpy(),
               grads.x0.cpu().numpy(), grads.goal.cpu().numpy(), grads.b_inst.cpu().numpy())

    plain = None
    if not args.no_plain:
        sub = b.subset(range(1000))
        pb = SegmentBatchGPU(sub, device="cuda:0")
        popts = _lib.default_opts()
        popts.plain = 1
        popts.store_for_backward = 0
        sx0 = torch.as_tensor(sub.x0, device=dev)
        sg = torch.as_tensor(sub.goal, device=dev)
        pout = pb.alloc_outputs()
        pb.solve(sx0, sg, opts=popts, out=pout)
        torch.cuda.synchronize()
        t = time.perf_counter()
        pb.solve(sx0, sg, opts=popts, out=pout)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        pst = pout.status.cpu().numpy()
        pk = pout.kkt.cpu().numpy()
        pc = int(((pst == 0) & (pk <= KKT_OK)).sum() + (pst == 1).sum())
        plain = {"solves_per_s": pc / tp, "sample": "first 1000 edges, FP64 iterations, one launch per instance",
                 "s_per_1000": tp}
        pb.close()

    extras = None
    if not args.no_extras:
        extras = extra_workloads(admm_iters=args.admm_iters, edges=b, main_opts=opts)

    cpu = None
    err = alt_err = None
    if not args.no_cpu_baseline:
        cpu, orc = cpu_baseline(b, gbar)
        err = errors_vs_oracle(b, orc, *main_np)
        alt_err = errors_vs_oracle(b, orc, *alt_np)
        alt_rec["error_vs_oracle"] = alt_err

    rec = {
        "metric": "segment-QP solves/s at KKT res <=1e-6, fwd+bwd (fwd, plain and % roofline alongside)",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "edges50k_p7_clutter", "instances": b.n, "degree": 7, "faces": "8-24",
                   "reach_rows": 32, "admm_iters": int(opts.admm_iters), "rho": round(float(opts.rho), 6),
                   "schedule": int(opts.schedule), "launch_shape": int(opts.launch_shape),
                   "options": "autotuned" if tuned is not None else "fixed", "tuning": tuned,
                   "obstacles": 200, "polytopes": 2000, "launch": launch},
        "roofline": roof,
        "error_vs_oracle": err,
        "other_precision_form": alt_rec,
        "fwd_solves_per_s": counted / t_solve,
        "bwd_ms": t_bwd * 1e3,
        "counts": {"solved_kkt_ok": n_ok, "infeasible_certified": n_inf, "other": int(b.n - counted)},
        "polish_steps_mean": float(iters[:, 1].mean()),
        "plain": plain,
        "vs_plain": (value / plain["solves_per_s"]) if plain else None,
        "fwd_vs_plain": ((counted / t_solve) / plain["solves_per_s"]) if plain else None,
        "cpu_baseline": cpu,
        "other_workloads": extras,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
