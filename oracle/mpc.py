"""FP64 CPU reference for the MPC refinement QP (eq. MPC, Sec. III-D), one
instance at a time.  Test infrastructure only: imported by tests/ and the
CPU-baseline leg of bench.py, never by the library.

Model (the reduced-order model of Sec. II with gamma = 2 in R^3): state
x = (position p, velocity v), input u = acceleration, exact zero-order-hold
discretisation over the step dt:

    x_{k+1} = A x_k + B u_k,   A = [[I, dt I], [0, I]],   B = [[dt^2/2 I], [dt I]].

Problem over the horizon k = 0..N (readings of the garbled cost and of the
initial-condition set are listed with the design notes):

    minimise   sum_{k=1}^{N-1} (x_k - r_k)^T Q (x_k - r_k)
             + sum_{k=0}^{N-1} u_k^T R u_k + w |p_{k+1} - p_k|^2
    subject to x_{k+1} = A x_k + B u_k            (dynamics)
               x_0 = x0                           (start state)
               F1 x_k + F2 x_{k+1} <= G           (reachable rows, Thm. 2)
               n_k . P_j(x_k, x_{k+1}) >= l_k     (keep-out plane of step k,
                                                   j = 0..3)
               x_N = r_N                          (terminal state)

P_j(x_k, x_{k+1}) are the control points of the unique cubic Bezier curve on
[0, dt] joining the two full states (Lemma 1 with p = 2 gamma - 1 = 3):
P_0 = p_k, P_1 = p_k + dt/3 v_k, P_2 = p_{k+1} - dt/3 v_{k+1}, P_3 = p_{k+1}.
By the convex-hull property (Property 1) the plane rows keep the whole step
on the free side.

The variable is y = [x_0..x_N, u_0..u_{N-1}, c] with c = 1 fixed by an
equality, so the cost (linear terms included) is the quadratic form y^T M y
and the problem goes to the pinned dense solver of ``qp`` (phase-1 LP, then
the primal active-set method) unchanged.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
from scipy.optimize import linprog

from . import qp as _qp


def dynamics(dt: float):
    """Exact discretisation of p' = v, v' = u under a constant input."""
    I3 = np.eye(3)
    A = np.block([[I3, dt * I3], [np.zeros((3, 3)), I3]])
    B = np.vstack([0.5 * dt * dt * I3, dt * I3])
    return A, B


def cubic_points(xk, xk1, dt):
    """Control points (4 x 3) of the cubic Bezier curve on [0, dt] with
    b(0) = p_k, b'(0) = v_k, b(dt) = p_{k+1}, b'(dt) = v_{k+1} (Lemma 1)."""
    return np.array([xk[:3], xk[:3] + dt / 3.0 * xk[3:], xk1[:3] - dt / 3.0 * xk1[3:], xk1[:3]])


@dataclass
class MpcQP:
    N: int
    M: np.ndarray      # quadratic form of the cost over y
    A: np.ndarray      # inequality rows
    u: np.ndarray
    E: np.ndarray      # equality rows
    e: np.ndarray
    ix: int            # offset of x_0 in y
    iu: int            # offset of u_0 in y
    ic: int            # index of the constant 1

    def split(self, y):
        X = y[self.ix:self.ix + 6 * (self.N + 1)].reshape(self.N + 1, 6)
        U = y[self.iu:self.iu + 3 * self.N].reshape(self.N, 3)
        return X, U


def build(inst: dict) -> MpcQP:
    N, dt = int(inst["N"]), float(inst["dt"])
    Q, R, w = np.asarray(inst["Q"], float), np.asarray(inst["R"], float), float(inst["w"])
    F1, F2, G = np.asarray(inst["F1"], float), np.asarray(inst["F2"], float), np.asarray(inst["G"], float)
    x0, ref, planes = np.asarray(inst["x0"], float), np.asarray(inst["ref"], float), np.asarray(inst["planes"], float)
    Ad, Bd = dynamics(dt)
    nx = 6 * (N + 1)
    n = nx + 3 * N + 1
    ix, iu, ic = 0, nx, nx + 3 * N
    X = lambda k: slice(ix + 6 * k, ix + 6 * k + 6)
    P = lambda k: slice(ix + 6 * k, ix + 6 * k + 3)
    U = lambda k: slice(iu + 3 * k, iu + 3 * k + 3)

    # cost as y^T M y
    M = np.zeros((n, n))
    for k in range(1, N):
        Qr = Q @ ref[k]
        M[X(k), X(k)] += Q
        M[X(k), ic] -= Qr
        M[ic, X(k)] -= Qr
        M[ic, ic] += ref[k] @ Qr
    for k in range(N):
        M[U(k), U(k)] += R
        D = np.zeros((3, n))          # p_{k+1} - p_k
        D[:, P(k + 1)] = np.eye(3)
        D[:, P(k)] -= np.eye(3)
        M += w * D.T @ D

    # equalities: x_0 = x0, dynamics, x_N = r_N, c = 1
    E = np.zeros((6 + 6 * N + 6 + 1, n))
    e = np.zeros(E.shape[0])
    E[0:6, X(0)] = np.eye(6); e[0:6] = x0
    for k in range(N):
        r = slice(6 + 6 * k, 12 + 6 * k)
        E[r, X(k + 1)] = np.eye(6)
        E[r, X(k)] = -Ad
        E[r, U(k)] = -Bd
    E[6 + 6 * N:12 + 6 * N, X(N)] = np.eye(6); e[6 + 6 * N:12 + 6 * N] = ref[N]
    E[-1, ic] = 1.0; e[-1] = 1.0

    # inequalities: reachable rows, then the four plane rows of every step
    m = G.shape[0]
    rows, rhs = [], []
    for k in range(N):
        Rk = np.zeros((m, n))
        Rk[:, X(k)] = F1
        Rk[:, X(k + 1)] = F2
        rows.append(Rk); rhs.append(G.copy())
    # P_j = a_j p_k + b_j v_k + c_j p_{k+1} + d_j v_{k+1}, read off cubic_points
    # (linear in the two states) on unit states along the first axis
    e_p, e_v, z = np.eye(6)[0], np.eye(6)[3], np.zeros(6)
    coef = list(zip(cubic_points(e_p, z, dt)[:, 0], cubic_points(e_v, z, dt)[:, 0],
                    cubic_points(z, e_p, dt)[:, 0], cubic_points(z, e_v, dt)[:, 0]))
    for k in range(N):
        nk, lk = planes[k, :3], planes[k, 3]
        Rk = np.zeros((4, n))
        for j, (a, b, c, d) in enumerate(coef):
            Rk[j, P(k)] -= a * nk
            Rk[j, ix + 6 * k + 3:ix + 6 * k + 6] -= b * nk
            Rk[j, P(k + 1)] -= c * nk
            Rk[j, ix + 6 * (k + 1) + 3:ix + 6 * (k + 1) + 6] -= d * nk
        rows.append(Rk); rhs.append(np.full(4, -lk))
    return MpcQP(N=N, M=M, A=np.concatenate(rows), u=np.concatenate(rhs), E=E, e=e, ix=ix, iu=iu, ic=ic)


@dataclass
class MpcResult:
    status: int
    s_star: float
    X: np.ndarray          # (N+1) x 6, NaN unless optimal
    U: np.ndarray          # N x 3
    cost: float
    kkt: dict
    qp: MpcQP
    y: Optional[np.ndarray] = None
    mu: Optional[np.ndarray] = None
    nu: Optional[np.ndarray] = None
    W: Optional[list] = None


def feasible_box(inst: dict):
    """An outer box of every feasible point, from the instance's own rows.

    Relaxation: keep x_0 = x0, the dynamics and the reachable rows
    F1 x_k + F2 x_{k+1} <= G; drop the plane rows and the terminal state.
    Forward propagation over the steps: if x_k lies in the box B_k, then
    (x_k, u_k) satisfies (F1 + F2 A) x_k + F2 B u_k <= G, so u_k and
    x_{k+1} = A x_k + B u_k lie within the bounds of small LPs over
    (x_k, u_k) in B_k x R^3 with those rows (one LP per bound), and B_{k+1}
    is the box of x_{k+1}.  By induction every feasible y is in the boxes.
    Each LP bound is widened by 1e-7 (1 + |bound|) against the LP's own
    tolerances.  Returns (lo, hi) over y = [x_0..x_N, u_0..u_{N-1}, 1], or
    None when some bound is infinite (the rows leave the set unbounded)."""
    N, dt = int(inst["N"]), float(inst["dt"])
    F1, F2, G = np.asarray(inst["F1"], float), np.asarray(inst["F2"], float), np.asarray(inst["G"], float)
    Ad, Bd = dynamics(dt)
    x0 = np.asarray(inst["x0"], float)
    nx = 6 * (N + 1)
    lo = np.zeros(nx + 3 * N + 1)
    hi = np.zeros_like(lo)
    lo[:6] = hi[:6] = x0
    lo[-1] = hi[-1] = 1.0
    # stage rows over z = (x_k, u_k)
    Az = np.hstack([F1 + F2 @ Ad, F2 @ Bd])
    # objectives: u_k (3) and x_{k+1} = [A B] z (6)
    obj = np.vstack([np.hstack([np.zeros((3, 6)), np.eye(3)]), np.hstack([Ad, Bd])])
    xl, xh = x0.copy(), x0.copy()
    for k in range(N):
        bounds = [(float(a), float(b)) for a, b in zip(xl, xh)] + [(None, None)] * 3
        vlo, vhi = np.zeros(9), np.zeros(9)
        for j in range(9):
            for sgn in (1.0, -1.0):
                res = linprog(sgn * obj[j], A_ub=Az if Az.size else None, b_ub=G if Az.size else None,
                              bounds=bounds, method="highs")
                if res.status != 0:
                    return None
                v = sgn * float(res.fun)
                pad = 1e-7 * (1.0 + abs(v))
                if sgn > 0:
                    vlo[j] = v - pad
                else:
                    vhi[j] = v + pad
        lo[nx + 3 * k:nx + 3 * k + 3], hi[nx + 3 * k:nx + 3 * k + 3] = vlo[:3], vhi[:3]
        xl, xh = vlo[3:], vhi[3:]
        lo[6 * (k + 1):6 * (k + 2)], hi[6 * (k + 1):6 * (k + 2)] = xl, xh
    return lo, hi


def y_bound(inst: dict):
    """The bound the phase-1 Farkas check uses: ``feasible_box`` (None when
    the reachable rows leave the relaxed set unbounded; then no instance is
    certified infeasible)."""
    return feasible_box(inst)


def solve(inst: dict, tau: float = _qp.TAU) -> MpcResult:
    q = build(inst)
    N = q.N
    ph = _qp.phase1(q.A, q.u, q.E, q.e, lambda: y_bound(inst), tau)
    nanX, nanU = np.full((N + 1, 6), np.nan), np.full((N, 3), np.nan)
    if not ph.feasible:
        st = _qp.INFEASIBLE if ph.certified else _qp.UNCERTIFIED
        return MpcResult(st, ph.s, nanX, nanU, np.inf, {}, q)
    W0 = _qp.initial_working_set(q.A, q.u, q.E, ph.y)
    r = _qp.active_set(q.M, q.A, q.u, q.E, q.e, ph.y, W0)
    st = (_qp.SOLVED if ph.certified else _qp.UNCERTIFIED) if r.status == _qp.SOLVED else r.status
    X, U = q.split(r.y)
    return MpcResult(st, ph.s, X.copy(), U.copy(), _qp.objective(q.M, r.y), r.res, q, r.y, r.mu, r.nu, r.W)
