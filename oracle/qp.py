"""FP64 CPU reference solver for one convex QP (test infrastructure only).

    minimise  y^T Q y   subject to   A y <= u,   E y = e

Used for the segment problems of the paper's edge evaluation: each candidate
edge is a curve whose control points must stay in a free-space polytope
(Property 1) and in the reachable Bezier polytope of Theorem 2.  The paper
solves its small QPs with OSQP (Sec. IV); the oracle instead reaches the
exact optimum, in two plain steps:

1. ``phase1``: the LP  min s  s.t.  (a_r y - u_r)/|a_r| <= s,  E y = e,
   solved by the library LP solver (HiGHS through scipy).  Its value ``s*``
   classifies the instance (s* <= -tau feasible, s* >= tau infeasible, else
   uncertified); the returned interior point or Farkas vector is re-verified
   here in FP64 before it is trusted.
2. ``active_set``: the primal active-set method (Nocedal & Wright,
   Numerical Optimization, 2nd ed., Algorithm 16.3) started at the phase-1
   point, each equality-constrained subproblem solved by a dense KKT solve.

Nothing here is shared with the HIP path.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.optimize import linprog

TAU = 1e-4          # certified margin on the row-normalised phase-1 value

SOLVED, INFEASIBLE, MAXITER, POLISH_FAILED, NUMERICAL = 0, 1, 2, 3, 4
UNCERTIFIED = -1


@dataclass
class Phase1:
    s: float                  # optimal normalised violation
    y: Optional[np.ndarray]   # phase-1 point (feasible side)
    farkas_w: Optional[np.ndarray] = None   # >= 0, on the A rows
    farkas_nu: Optional[np.ndarray] = None  # on the E rows
    certified: bool = False
    feasible: bool = False
    verify_gap: float = 0.0


def phase1(A, u, E, e, y_bound, tau: float = TAU) -> Phase1:
    """Phase-1 LP with row-normalised violations, then an FP64 re-check of
    whichever certificate the LP hands back.

    ``y_bound`` encloses every feasible point, for the Farkas check: a scalar
    Y (|y|_inf <= Y), a pair of arrays (lo, hi) (lo <= y <= hi), or None
    when no bound is known (then infeasibility is never certified); or a
    function returning one of these, called only when the LP reports
    infeasibility."""
    m, n = A.shape
    nrm = np.linalg.norm(A, axis=1)
    An = A / nrm[:, None]
    un = u / nrm
    c = np.zeros(n + 1); c[-1] = 1.0
    A_ub = np.hstack([An, -np.ones((m, 1))])
    A_eq = np.hstack([E, np.zeros((E.shape[0], 1))])
    res = linprog(c, A_ub=A_ub, b_ub=un, A_eq=A_eq, b_eq=e,
                  bounds=[(None, None)] * (n + 1), method="highs")
    if res.status != 0:
        raise RuntimeError(f"phase-1 LP failed: {res.message}")
    s = float(res.fun)
    out = Phase1(s=s, y=None)
    if s < 0:
        y = res.x[:n].copy()
        # project onto {E y = e} so the equalities hold to rounding
        y -= E.T @ np.linalg.solve(E @ E.T, E @ y - e)
        viol = float(np.max((An @ y - un)))
        out.y = y
        out.feasible = True
        out.certified = s <= -tau and viol <= s + 1e-9
        out.verify_gap = -viol
    else:
        mu = np.maximum(-res.ineqlin.marginals, 0.0)
        nu = -res.eqlin.marginals
        w = mu / nrm
        r = A.T @ w + E.T @ nu
        gap = -(u @ w + e @ nu)
        # For any y with A y <= u, E y = e inside the bound:
        # r.y = w.Ay + nu.Ey <= u.w + e.nu = -gap, while r.y >= min over the
        # bound of r.y (-|r|_1 Y for a scalar Y); no such y exists when that
        # minimum exceeds -gap.
        if callable(y_bound):
            y_bound = y_bound()
        if y_bound is None:
            slack = -np.inf
        elif np.isscalar(y_bound):
            slack = gap - np.abs(r).sum() * float(y_bound)
        else:
            lo, hi = (np.asarray(a, float) for a in y_bound)
            slack = gap + float(np.sum(np.minimum(r * lo, r * hi)))
        out.farkas_w, out.farkas_nu = w, nu
        out.feasible = False
        out.verify_gap = float(slack / max(1.0, w.sum()))
        out.certified = s >= tau and slack > 0
    return out


@dataclass
class QPResult:
    y: np.ndarray
    mu: np.ndarray            # m, >= 0
    nu: np.ndarray            # |E|
    W: List[int]
    iters: int
    status: int
    res: dict = field(default_factory=dict)


def _eqp(Q2, A, E, e, u, W):
    """Minimiser of y^T Q y on {E y = e, A_W y = u_W} and its multipliers
    (grad f + C^T lam = 0 with C = [E; A_W])."""
    n = Q2.shape[0]
    C = np.vstack([E, A[W]]) if W else E
    d = np.concatenate([e, u[W]]) if W else e
    k = C.shape[0]
    K = np.zeros((n + k, n + k))
    K[:n, :n] = Q2
    K[:n, n:] = C.T
    K[n:, :n] = C
    rhs = np.concatenate([np.zeros(n), d])
    sol = np.linalg.solve(K, rhs)
    return sol[:n], sol[n:]


def initial_working_set(A, u, E, y0) -> List[int]:
    """Rows tight at the phase-1 point, kept linearly independent of the
    equality rows and of each other (none when the point is interior)."""
    slack = u - A @ y0
    W0: List[int] = []
    for i in np.where(slack <= 1e-12 * (1 + np.abs(u)))[0]:
        C = np.vstack([E, A[W0 + [int(i)]]])
        if np.linalg.matrix_rank(C) == C.shape[0]:
            W0.append(int(i))
    return W0


def active_set(Q, A, u, E, e, y0, W0=(), max_iter: Optional[int] = None) -> QPResult:
    """Primal active-set method (N&W Alg. 16.3) for min y^T Q y, A y <= u,
    E y = e, from a feasible ``y0`` with working set ``W0`` (inequality rows
    that are tight at ``y0`` and linearly independent)."""
    Q2 = 2.0 * Q
    m = A.shape[0]
    ne = E.shape[0]
    y = np.array(y0, dtype=np.float64, copy=True)
    W = list(W0)
    max_iter = max_iter or 20 * max(m, 1)
    zero_steps = 0
    bland = False
    anorm = np.linalg.norm(A, axis=1)
    for it in range(1, max_iter + 1):
        x, lam = _eqp(Q2, A, E, e, u, W)
        p = x - y
        pn = np.max(np.abs(p))
        if pn <= 1e-10 * (1.0 + np.max(np.abs(y))):
            alpha, block = 1.0, -1
        else:
            Ap = A @ p
            slack = u - A @ y
            alpha, block = 1.0, -1
            inW = np.zeros(m, bool); inW[W] = True
            cand = np.where((~inW) & (Ap > 1e-12 * anorm * pn))[0]
            if cand.size:
                ratios = np.maximum(slack[cand], 0.0) / Ap[cand]
                rmin = ratios.min()
                if rmin < 1.0:
                    ties = cand[ratios <= rmin + 1e-15 * max(1.0, rmin)]
                    alpha, block = float(rmin), int(ties.min())
        if block < 0:
            y = x
            zero_steps = 0
            mu_W = lam[ne:]
            if mu_W.size == 0:
                return _finish(Q, A, u, E, e, y, W, lam, it, SOLVED)
            tol = 1e-11 * (1.0 + np.max(np.abs(lam)))
            neg = np.where(mu_W < -tol)[0]
            if neg.size == 0:
                return _finish(Q, A, u, E, e, y, W, lam, it, SOLVED)
            if bland:
                drop = int(min(neg, key=lambda q: W[q]))
            else:
                mn = mu_W.min()
                ties = [q for q in neg if mu_W[q] <= mn + 1e-15 * abs(mn)]
                drop = int(min(ties, key=lambda q: W[q]))
            W.pop(drop)
        else:
            y = y + alpha * p
            W.append(block)
            zero_steps = zero_steps + 1 if alpha <= 1e-15 else 0
            if zero_steps >= 50:
                bland = True
    x, lam = _eqp(Q2, A, E, e, u, W)
    return _finish(Q, A, u, E, e, y, W, lam, max_iter, MAXITER)


def _finish(Q, A, u, E, e, y, W, lam, iters, status) -> QPResult:
    ne = E.shape[0]
    mu = np.zeros(A.shape[0])
    mu[W] = lam[ne:]
    nu = lam[:ne].copy()
    r = QPResult(y=y, mu=mu, nu=nu, W=sorted(W), iters=iters, status=status)
    r.res = kkt_residuals(Q, A, u, E, e, y, mu, nu)
    return r


def kkt_residuals(Q, A, u, E, e, y, mu, nu) -> dict:
    """Scaled KKT residuals of a candidate (y, mu, nu) for
    min y^T Q y, A y <= u, E y = e (stationarity 2Qy + A^T mu + E^T nu = 0)."""
    Ay = A @ y
    g = 2.0 * Q @ y
    ATmu = A.T @ mu
    ETnu = E.T @ nu
    inf = lambda v: float(np.max(np.abs(v))) if np.size(v) else 0.0
    prim_in = inf(np.maximum(Ay - u, 0.0)) / (1.0 + max(inf(Ay), inf(u)))
    prim_eq = inf(E @ y - e) / (1.0 + inf(e))
    dual = inf(g + ATmu + ETnu) / (1.0 + max(inf(g), inf(ATmu), inf(ETnu)))
    mun = inf(mu)
    comp = float(np.max(mu * np.abs(u - Ay))) / (1.0 + mun) if mu.size else 0.0
    dsign = float(np.max(np.maximum(-mu, 0.0))) / (1.0 + mun) if mu.size else 0.0
    return dict(prim_in=prim_in, prim_eq=prim_eq, dual=dual, comp=comp, dual_sign=dsign,
                max=max(prim_in, prim_eq, dual, comp, dsign))


def objective(Q, y) -> float:
    return float(y @ Q @ y)
