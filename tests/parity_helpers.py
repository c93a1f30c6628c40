"""Shared helpers of the GPU parity tests: run the oracle on the same seeded
instances and compare element by element with the stated tolerances.

Tolerances (per result):
  status    bit-exact where the oracle certifies the class (|s*| >= 1e-4)
  cost      |f - f_or| <= 1e-6 |f_or| + 1e-9
  P*        |P - P_or|_inf <= 1e-6 (1 + |P_or|_inf)
  KKT       scaled residual <= 1e-6
  gradients |g - g_or|_2 <= 1e-4 max(|g_or|_2, 1e-8)
"""
from __future__ import annotations

import multiprocessing as mp
from typing import Sequence

import numpy as np

from oracle import qp, segment
from workloads import gen

COST_RTOL, COST_ATOL = 1e-6, 1e-9
P_TOL = 1e-6
KKT_TOL = 1e-6
GRAD_RTOL = 1e-4


def _oracle_one(inst):
    r = segment.solve(inst)
    return dict(status=r.status, cost=r.cost, P=r.P, s=r.s_star, certified=r.certified)


def oracle_batch(batch: gen.SegmentBatch, idx: Sequence[int] = None, workers: int = 8):
    idx = range(batch.n) if idx is None else idx
    insts = [batch.instance(i) for i in idx]
    if len(insts) < 16:
        return [_oracle_one(x) for x in insts]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_oracle_one, insts, chunksize=8)


def compare(batch, gpu_P, gpu_cost, gpu_status, gpu_kkt, idx=None, label=""):
    """Compare GPU outputs (numpy, full batch) with the oracle on ``idx``;
    returns a dict of error figures and asserts the tolerances."""
    idx = list(range(batch.n)) if idx is None else list(idx)
    orc = oracle_batch(batch, idx)
    pt_off = np.concatenate([[0], np.cumsum(batch.degree.astype(np.int64) + 1)])
    n_cert = n_solved = 0
    cost_err = p_err = kkt_max = 0.0
    mism = []
    for k, i in enumerate(idx):
        o = orc[k]
        st = int(gpu_status[i])
        if o["status"] in (qp.SOLVED, qp.INFEASIBLE):
            n_cert += 1
            if st != o["status"]:
                mism.append((i, o["status"], st, o["s"]))
                continue
        if o["status"] == qp.SOLVED and st == qp.SOLVED:
            n_solved += 1
            Pg = gpu_P[3 * pt_off[i]:3 * pt_off[i + 1]].reshape(-1, 3)
            ce = abs(gpu_cost[i] - o["cost"])
            assert ce <= COST_RTOL * abs(o["cost"]) + COST_ATOL, (label, i, gpu_cost[i], o["cost"])
            cost_err = max(cost_err, ce / (abs(o["cost"]) + COST_ATOL / COST_RTOL))
            pe = np.abs(Pg - o["P"]).max() / (1.0 + np.abs(o["P"]).max())
            assert pe <= P_TOL, (label, i, pe)
            p_err = max(p_err, pe)
            assert gpu_kkt[i] <= KKT_TOL, (label, i, gpu_kkt[i])
            kkt_max = max(kkt_max, float(gpu_kkt[i]))
        if o["status"] == qp.INFEASIBLE and st == qp.INFEASIBLE:
            assert np.isinf(gpu_cost[i])
    out = dict(label=label, n=len(idx), certified=n_cert, solved=n_solved, status_mismatches=mism,
               max_cost_rel_err=cost_err, max_P_err=p_err, max_kkt=kkt_max)
    print("parity", out, flush=True)
    assert not mism, mism[:10]
    return out
