"""Oracle rows of a multi-segment path (test infrastructure only).

A path is S degree-p segments joined with continuous position, velocity and
acceleration (equal durations, so the join conditions are C0, C1 and C2 on
the control points).  Each segment keeps its control points in its own
free-space polytope (Property 1), respects the velocity and acceleration
difference bounds, and satisfies its reachable Bezier polytope (Theorem 2)
from its own start state: the chain's start state for the first segment,
the join state ``(P^s_0, p/T (P^s_1 - P^s_0))`` for the others (linear in the
control points, so those rows move to the left-hand side).  The start point
and the goal point are pinned.  Solved by the same phase-1 LP and primal
active-set method as single segments (``oracle.qp``).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import bezier, qp


@dataclass
class ChainQP:
    S: int
    p: int
    Q: np.ndarray
    A: np.ndarray
    u: np.ndarray
    E: np.ndarray
    e: np.ndarray
    seg_of_row: np.ndarray


def build(ch: dict) -> ChainQP:
    p, T = ch["p"], ch["T"]
    vmax, amax = ch["vmax"], ch["amax"]
    segs = ch["segments"]
    S = len(segs)
    npt = p + 1
    nseg = 3 * npt
    n = S * nseg
    I3 = np.eye(3)
    Q = np.kron(np.eye(S), bezier.hessian(p, T))
    rows, rhs, sid = [], [], []
    D1 = p / T * np.kron(bezier.diff_matrix(p, 1), I3)
    D2 = p * (p - 1) / T ** 2 * np.kron(bezier.diff_matrix(p, 2), I3)
    for s, sg in enumerate(segs):
        off = s * nseg
        Af, bf = sg["A_face"], sg["b_face"]
        nf = Af.shape[0]
        for k in range(npt):
            R = np.zeros((nf, n))
            R[:, off + 3 * k:off + 3 * k + 3] = Af
            rows.append(R); rhs.append(bf); sid += [s] * nf
        for D, bound in ((D1, vmax), (D2, amax)):
            for sgn in (1.0, -1.0):
                R = np.zeros((D.shape[0], n))
                R[:, off:off + nseg] = sgn * D
                rows.append(R); rhs.append(np.full(D.shape[0], bound)); sid += [s] * D.shape[0]
        H, h0, G = sg["H"], sg["h0"], sg["G"]
        R = np.zeros((H.shape[0], n))
        R[:, off:off + nseg] = H
        if s == 0:
            b = h0 + G @ ch["x0"]
        else:
            # G x0_s with x0_s = (P_0, p/T (P_1 - P_0)) of this segment
            R[:, off:off + 3] -= G[:, :3]
            R[:, off + 3:off + 6] -= p / T * G[:, 3:]
            R[:, off:off + 3] += p / T * G[:, 3:]
            b = h0.copy()
        rows.append(R); rhs.append(b); sid += [s] * H.shape[0]
    A = np.concatenate(rows)
    u = np.concatenate(rhs)
    E, e = [], []

    def sel(s, k):
        M = np.zeros((3, n))
        M[:, s * nseg + 3 * k:s * nseg + 3 * k + 3] = I3
        return M

    E.append(sel(0, 0)); e.append(ch["x0"][:3])
    E.append(sel(S - 1, p)); e.append(ch["goal"])
    for s in range(S - 1):
        a, b_ = s, s + 1
        E.append(sel(a, p) - sel(b_, 0)); e.append(np.zeros(3))
        E.append((sel(a, p) - sel(a, p - 1)) - (sel(b_, 1) - sel(b_, 0))); e.append(np.zeros(3))
        E.append((sel(a, p) - 2 * sel(a, p - 1) + sel(a, p - 2))
                 - (sel(b_, 2) - 2 * sel(b_, 1) + sel(b_, 0))); e.append(np.zeros(3))
    return ChainQP(S=S, p=p, Q=Q, A=A, u=u, E=np.concatenate(E), e=np.concatenate(e),
                   seg_of_row=np.asarray(sid))


@dataclass
class ChainResult:
    status: int
    s_star: float
    certified: bool
    P: Optional[np.ndarray]      # S x (p+1) x 3
    cost: float
    kkt: dict
    qp: ChainQP


def y_bound(ch: dict) -> float:
    """Consecutive control points of the joined polygon differ by at most
    vmax T / p per axis, so every point is within S vmax T of the start."""
    return float(np.max(np.abs(ch["x0"][:3])) + len(ch["segments"]) * ch["vmax"] * ch["T"] + 1.0)


def solve(ch: dict, tau: float = qp.TAU) -> ChainResult:
    c = build(ch)
    ph = qp.phase1(c.A, c.u, c.E, c.e, y_bound(ch), tau)
    shape = (c.S, c.p + 1, 3)
    if not ph.feasible:
        return ChainResult(qp.INFEASIBLE if ph.certified else qp.UNCERTIFIED, ph.s, ph.certified,
                           np.full(shape, np.nan), np.inf, {}, c)
    r = qp.active_set(c.Q, c.A, c.u, c.E, c.e, ph.y, qp.initial_working_set(c.A, c.u, c.E, ph.y))
    st = (qp.SOLVED if ph.certified else qp.UNCERTIFIED) if r.status == qp.SOLVED else r.status
    return ChainResult(st, ph.s, ph.certified, r.y.reshape(shape), qp.objective(c.Q, r.y), r.res, c)
