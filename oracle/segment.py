"""Per-instance oracle for the segment problem and its derivatives.

``solve(inst)`` builds the dense rows (``rows.build``), classifies the
instance with the phase-1 LP, and on the feasible side runs the primal
active-set method to the exact optimum.  ``gradients`` differentiates the
optimum with respect to the start state ``x0``, the goal waypoint and the
free-space offsets ``b``:

* optimal cost, by the envelope theorem: with the Lagrangian
  ``L = y^T Q y + mu^T (A y - u(theta)) + nu^T (E y - e(theta))``,
  ``df*/dtheta = -mu^T du/dtheta - nu^T de/dtheta``;
* optimal solution, by implicit differentiation of the KKT system on the
  optimal active set ``W``: ``K_W [w; omega] = [gbar; 0]`` with
  ``K_W = [2Q C^T; C 0]``, ``C = [E; A_W]``, then
  ``d(gbar.y*)/dtheta = omega^T d[e; u_W]/dtheta``.

This is test infrastructure; the product path never imports it.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import qp as _qp
from . import rows as _rows


@dataclass
class SegmentResult:
    status: int                 # qp.SOLVED / qp.INFEASIBLE / qp.UNCERTIFIED / qp.MAXITER
    s_star: float
    certified: bool
    P: Optional[np.ndarray]     # (p+1) x 3, NaN when infeasible
    cost: float
    mu: Optional[np.ndarray]
    nu: Optional[np.ndarray]
    W: Optional[list]
    kkt: dict
    qp: _rows.SegmentQP
    iters: int = 0


def y_bound(inst: dict) -> float:
    """Every feasible point satisfies |P_k - P_0|_inf <= k vmax T / p, so
    |y|_inf <= |pos0|_inf + vmax T."""
    return float(np.max(np.abs(inst["x0"][:3])) + inst["vmax"] * inst["T"] + 1.0)


def solve(inst: dict, tau: float = _qp.TAU) -> SegmentResult:
    q = _rows.build(inst)
    ph = _qp.phase1(q.A, q.u, q.E, q.e, y_bound(inst), tau)
    if not ph.feasible:
        st = _qp.INFEASIBLE if ph.certified else _qp.UNCERTIFIED
        return SegmentResult(st, ph.s, ph.certified, np.full((q.p + 1, 3), np.nan), np.inf,
                             None, None, None, {}, q)
    W0 = _qp.initial_working_set(q.A, q.u, q.E, ph.y)
    r = _qp.active_set(q.Q, q.A, q.u, q.E, q.e, ph.y, W0)
    if r.status == _qp.SOLVED:
        st = _qp.SOLVED if ph.certified else _qp.UNCERTIFIED
    else:
        st = r.status
    return SegmentResult(st, ph.s, ph.certified,
                         r.y.reshape(q.p + 1, 3), _qp.objective(q.Q, r.y), r.mu, r.nu, r.W,
                         r.res, q, r.iters)


def is_solved(res: SegmentResult) -> bool:
    """An optimum was reached (certified or not)."""
    return res.mu is not None and res.kkt.get("max", 1.0) <= 1e-9


@dataclass
class Gradients:
    cost_x0: np.ndarray
    cost_goal: np.ndarray
    cost_b: np.ndarray
    sol_x0: np.ndarray
    sol_goal: np.ndarray
    sol_b: np.ndarray

    def combined(self, gf: float):
        """Gradients of ``gbar.P* + gf * f*``."""
        return (self.sol_x0 + gf * self.cost_x0, self.sol_goal + gf * self.cost_goal,
                self.sol_b + gf * self.cost_b)


def gradients(res: SegmentResult, gbar: Optional[np.ndarray] = None) -> Gradients:
    """Envelope-theorem cost gradient and KKT-adjoint solution VJP on the
    optimal active set of an optimised instance."""
    q = res.qp
    n = q.n
    mu, nu = res.mu, res.nu
    cost_x0 = -(q.du_dx0.T @ mu) - q.de_dx0.T @ nu
    cost_goal = -(q.de_dg.T @ nu)
    cost_b = -(q.du_db.T @ mu)
    if gbar is None:
        gbar = np.zeros(n)
    W = list(res.W)
    C = np.vstack([q.E, q.A[W]]) if W else q.E
    k = C.shape[0]
    K = np.zeros((n + k, n + k))
    K[:n, :n] = 2.0 * q.Q
    K[:n, n:] = C.T
    K[n:, :n] = C
    sol = np.linalg.solve(K, np.concatenate([np.asarray(gbar, float).ravel(), np.zeros(k)]))
    om = sol[n:]
    om_e, om_w = om[:q.E.shape[0]], om[q.E.shape[0]:]
    sol_x0 = q.de_dx0.T @ om_e + (q.du_dx0[W].T @ om_w if W else 0.0)
    sol_goal = q.de_dg.T @ om_e
    sol_b = q.du_db[W].T @ om_w if W else np.zeros(q.du_db.shape[1])
    return Gradients(cost_x0, cost_goal, cost_b, np.asarray(sol_x0, float) * np.ones(6),
                     sol_goal, np.asarray(sol_b, float) * np.ones(q.du_db.shape[1]))


def margins(res: SegmentResult) -> dict:
    """Degeneracy measures used to pick instances whose gradients are
    well defined: LICQ ratio of the active rows, smallest active multiplier
    and smallest normalised inactive slack."""
    q = res.qp
    W = list(res.W)
    C = np.vstack([q.E, q.A[W]]) if W else q.E
    sv = np.linalg.svd(C, compute_uv=False)
    licq = float(sv.min() / sv.max())
    mu_inf = float(np.max(np.abs(res.mu))) if res.mu.size else 0.0
    min_mu = float(np.min(res.mu[W])) / max(1.0, mu_inf) if W else np.inf
    y = res.P.ravel()
    inact = np.setdiff1d(np.arange(q.m), W)
    nrm = np.linalg.norm(q.A, axis=1)
    sl = (q.u - q.A @ y) / nrm
    min_slack = float(sl[inact].min()) if inact.size else np.inf
    return dict(licq=licq, min_mu=min_mu, min_slack=min_slack)


def gradient_certified(res: SegmentResult, thr: float = 1e-4) -> bool:
    if not is_solved(res) or not res.certified:
        return False
    mg = margins(res)
    return mg["licq"] >= 1e-8 and mg["min_mu"] >= thr and mg["min_slack"] >= thr


def perturbed(inst: dict, which: str, j: int, h: float) -> dict:
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in inst.items()}
    if which == "x0":
        out["x0"][j] += h
    elif which == "goal":
        out["goal"][j] += h
    elif which == "b":
        out["b_face"][j] += h
    else:
        raise ValueError(which)
    return out


def fd_gradients(inst: dict, gbar: np.ndarray, gf: float, h: float = 1e-6):
    """Central finite differences of ``gbar.P* + gf f*`` by re-solving."""
    def loss(ii):
        r = solve(ii)
        return float(np.dot(gbar.ravel(), r.P.ravel()) + gf * r.cost)
    out = {}
    for which, size in (("x0", 6), ("goal", 3), ("b", inst["b_face"].shape[0])):
        g = np.zeros(size)
        for j in range(size):
            g[j] = (loss(perturbed(inst, which, j, h)) - loss(perturbed(inst, which, j, -h))) / (2 * h)
        out[which] = g
    return out
