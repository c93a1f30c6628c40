"""Pins of the FP64 oracle QP (constraint rows, phase 1, active set).

The segment problem is the per-edge curve of the paper's Bezier graph
(Sec. III) with the free-space faces lifted to every control point
(Property 1), the reachable polytope of Theorem 2 and difference-operator
bounds.  The pins are independent of the oracle's own solver:
brute-force active-set enumeration, textbook special cases (straight line,
Hermite interpolation of Lemma 1), scipy's SLSQP, curve sampling with
numpy's polynomial arithmetic, and translation invariance."""
import itertools

import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly
from scipy.optimize import linprog, minimize

from oracle import bezier, qp, rows, segment
from workloads import gen


# ---------------------------------------------------------------- brute force
def tiny_problem(seed, d, p, m):
    """min y^T Q y with Q the Bezier energy in R^d, both end points pinned,
    m random inequality rows around a random feasible point."""
    rng = np.random.default_rng(seed)
    n = d * (p + 1)
    Q = bezier.hessian(p, 1.0, d)
    y_feas = rng.uniform(-1, 1, n)
    E = np.zeros((2 * d, n))
    E[:d, :d] = np.eye(d)
    E[d:, -d:] = np.eye(d)
    e = E @ y_feas
    A = rng.standard_normal((m, n))
    u = A @ y_feas + rng.uniform(0.0, 0.5, m)
    return Q, A, u, E, e, y_feas


def brute_force(Q, A, u, E, e):
    """Enumerate every working set; return the KKT points."""
    n = Q.shape[0]
    m = A.shape[0]
    pts = []
    for k in range(0, min(m, n - E.shape[0]) + 1):
        for W in itertools.combinations(range(m), k):
            C = np.vstack([E, A[list(W)]])
            if np.linalg.matrix_rank(C) < C.shape[0]:
                continue
            K = np.block([[2 * Q, C.T], [C, np.zeros((C.shape[0], C.shape[0]))]])
            rhs = np.concatenate([np.zeros(n), e, u[list(W)]])
            sol = np.linalg.solve(K, rhs)
            y, lam = sol[:n], sol[n:]
            mu = lam[E.shape[0]:]
            if np.all(A @ y <= u + 1e-10) and np.all(mu >= -1e-10):
                pts.append(y)
    return pts


@pytest.mark.parametrize("seed", range(12))
def test_active_set_matches_brute_force(seed):
    d = 1 + seed % 2
    p = 3 + (seed // 2) % 2
    m = 6 + seed % 7
    Q, A, u, E, e, y0 = tiny_problem(seed, d, p, m)
    kkt_pts = brute_force(Q, A, u, E, e)
    assert kkt_pts, "a feasible strictly convex problem has a KKT point"
    ref = kkt_pts[0]
    for y in kkt_pts[1:]:   # strictly convex on the feasible set: unique
        assert np.allclose(y, ref, atol=1e-9)
    r = qp.active_set(Q, A, u, E, e, y0, [i for i in range(m) if abs(A[i] @ y0 - u[i]) < 1e-14])
    assert r.status == qp.SOLVED
    assert np.max(np.abs(r.y - ref)) <= 1e-10 * (1 + np.abs(ref).max())
    assert r.res["max"] <= 1e-12


# ------------------------------------------------------------ special cases
def line_instance(p=7, T=1.0, seed=0):
    """Loose constraints: the straight constant-speed line is feasible."""
    rng = np.random.default_rng(seed)
    x0 = np.concatenate([rng.uniform(4, 6, 3), rng.uniform(-1, 1, 3)])
    g = x0[:3] + rng.uniform(-1, 1, 3)
    r = 8
    H = rng.standard_normal((r, 3 * (p + 1)))
    H /= np.linalg.norm(H, axis=1, keepdims=True)
    return dict(p=p, T=T, vmax=10.0, amax=10.0,
                A_face=np.concatenate([np.eye(3), -np.eye(3)]),
                b_face=np.concatenate([np.full(3, 20.0), np.full(3, 20.0)]),
                H=H, h0=np.full(r, 1e3), G=np.zeros((r, 6)), x0=x0, goal=g)


@pytest.mark.parametrize("p", [3, 5, 7, 9])
def test_straight_line_special_case(p):
    inst = line_instance(p=p, seed=p)
    res = segment.solve(inst)
    assert res.status == qp.SOLVED
    k = np.arange(p + 1)[:, None] / p
    line = inst["x0"][:3] + k * (inst["goal"] - inst["x0"][:3])
    assert abs(res.cost) <= 1e-9
    assert np.max(np.abs(res.P - line)) <= 1e-9


def test_hermite_special_case_lemma1():
    """Lemma 1 at the minimal degree p = 3: with position and velocity
    pinned at both ends the curve is unique (cubic Hermite:
    P_1 = P_0 + T v_0 / 3, P_2 = P_3 - T v_T / 3), and so is the QP."""
    rng = np.random.default_rng(11)
    p, T = 3, 0.8
    P0, P3 = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    v0, vT = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
    P1 = P0 + T * v0 / 3
    P2 = P3 - T * vT / 3
    n = 12
    Q = bezier.hessian(p, T)
    E = np.eye(n)
    e = np.concatenate([P0, P1, P2, P3])
    A = np.zeros((1, n))
    A[0, 0] = 1.0
    u = np.array([P0[0] + 1.0])
    r = qp.active_set(Q, A, u, E, e, e.copy())
    assert np.allclose(r.y, e, atol=1e-14)
    a, c = P2 - 2 * P1 + P0, P3 - 2 * P2 + P1
    assert abs(qp.objective(Q, r.y) - 36 / T ** 3 * (a @ a + a @ c + c @ c) / 3) <= 1e-12


def test_far_goal_is_infeasible():
    """Every velocity row bounds |P_{k+1} - P_k| by vmax T / p per axis, so a
    goal more than vmax T away along an axis cannot be reached."""
    inst = line_instance(p=7, seed=3)
    inst["vmax"] = 1.0
    inst["goal"] = inst["x0"][:3] + np.array([1.2, 0.0, 0.0])
    res = segment.solve(inst)
    assert res.status == qp.INFEASIBLE and res.certified
    inst["goal"] = inst["x0"][:3] + np.array([0.8, 0.0, 0.0])
    assert segment.solve(inst).status == qp.SOLVED


# ------------------------------------------------------------ row structure
def test_row_counts_cfg0():
    q = rows.build(gen.gen_cfg0(indices=[0]).instance(0))
    assert rows.row_counts(q) == {"face": 48, "vel": 42, "acc": 36, "reach": 32}


def _curve_checks(inst, P, tol=1e-9):
    T = inst["T"]
    t = np.linspace(0, T, 1001)
    pts = bezier.curve_bernstein(P, t, T)
    assert np.all(pts @ inst["A_face"].T <= inst["b_face"] + tol)
    # derivatives from numpy's power basis, not from the oracle's operators
    from tests.test_bezier import power_basis
    polys = power_basis(P, T)
    vel = np.stack([npoly.polyval(t, npoly.polyder(c, 1)) for c in polys], 1)
    acc = np.stack([npoly.polyval(t, npoly.polyder(c, 2)) for c in polys], 1)
    assert np.abs(vel).max() <= inst["vmax"] + 1e-7
    assert np.abs(acc).max() <= inst["amax"] + 1e-7
    return np.abs(vel).max(), np.abs(acc).max()


def test_solutions_satisfy_sampled_curve_invariants():
    """Property 1 applied to the curve and its derivative curves: the
    sampled curve stays in the polytope and within the derivative bounds.
    Some optima touch the bounds, so a wrong derivative scaling in the rows
    shows up as a violation here."""
    b = gen.gen_cfg0(64)
    vmaxes, amaxes = [], []
    for i in range(b.n):
        inst = b.instance(i)
        res = segment.solve(inst)
        if res.status == qp.SOLVED:
            v, a = _curve_checks(inst, res.P)
            vmaxes.append(v); amaxes.append(a)
            assert np.allclose(res.P[0], inst["x0"][:3], atol=1e-12)
            assert np.allclose(res.P[-1], inst["goal"], atol=1e-12)
    # some optimum must press on a derivative bound for the check to bite
    assert max(vmaxes) > 0.9 * b.vmax or max(amaxes) > 0.9 * b.amax


def test_derivative_rows_equal_end_derivatives():
    """The k = 0 velocity and acceleration rows give b'(0) and b''(0)."""
    inst = gen.gen_cfg0(indices=[3]).instance(0)
    q = rows.build(inst)
    rng = np.random.default_rng(0)
    P = rng.standard_normal((inst["p"] + 1, 3))
    from tests.test_bezier import power_basis
    polys = power_basis(P, inst["T"])
    v0 = np.array([npoly.polyval(0.0, npoly.polyder(c, 1)) for c in polys])
    a0 = np.array([npoly.polyval(0.0, npoly.polyder(c, 2)) for c in polys])
    vals = q.A @ P.ravel()
    vel = vals[q.kind == rows.VEL][:3]
    acc = vals[q.kind == rows.ACC][:3]
    assert np.allclose(vel, v0, atol=1e-10)
    assert np.allclose(acc, a0, atol=1e-9)


def test_translation_invariance():
    """The cost only sees second differences, so moving the pins, the
    polytope and the reachable rows (right-hand side re-expressed for the
    moved start state) by one vector moves the optimum by that vector."""
    inst = gen.gen_cfg0(indices=[1]).instance(0)
    base = segment.solve(inst)
    shift = np.array([3.0, -2.0, 5.0])
    moved = dict(inst)
    moved["x0"] = inst["x0"] + np.concatenate([shift, np.zeros(3)])
    moved["goal"] = inst["goal"] + shift
    moved["b_face"] = inst["b_face"] + inst["A_face"] @ shift
    p = inst["p"]
    # literal frame: h = h0 + G x0 must not change for the shifted rows
    moved["h0"] = inst["h0"] + inst["H"] @ np.tile(shift, p + 1) - inst["G"][:, :3] @ shift
    res = segment.solve(moved)
    assert res.status == base.status
    if base.status == qp.SOLVED:
        assert np.allclose(res.P, base.P + shift, atol=1e-9)
        assert abs(res.cost - base.cost) <= 1e-9 * (1 + abs(base.cost))


# ------------------------------------------------------------ phase 1 / KKT
def test_phase1_value_matches_other_lp_method():
    b = gen.gen_cfg0(16)
    for i in range(b.n):
        q = rows.build(b.instance(i))
        ph = qp.phase1(q.A, q.u, q.E, q.e, 100.0)
        m, n = q.A.shape
        nrm = np.linalg.norm(q.A, axis=1)
        res = linprog(np.r_[np.zeros(n), 1.0], A_ub=np.hstack([q.A / nrm[:, None], -np.ones((m, 1))]),
                      b_ub=q.u / nrm, A_eq=np.hstack([q.E, np.zeros((6, 1))]), b_eq=q.e,
                      bounds=[(None, None)] * (n + 1), method="highs-ipm")
        assert abs(res.fun - ph.s) <= 1e-7
        assert ph.certified


def test_certificates_verify():
    b = gen.gen_cfg1(indices=range(60))
    n_inf = 0
    for i in range(b.n):
        res = segment.solve(b.instance(i))
        if res.status == qp.INFEASIBLE:
            n_inf += 1
            q = res.qp
            ph = qp.phase1(q.A, q.u, q.E, q.e, segment.y_bound(b.instance(i)))
            w, nu = ph.farkas_w, ph.farkas_nu
            assert np.all(w >= 0)
            assert np.abs(q.A.T @ w + q.E.T @ nu).max() <= 1e-9 * (1 + np.abs(w).max())
            assert q.u @ w + q.e @ nu < -1e-6
        elif res.status == qp.SOLVED:
            assert res.kkt["max"] <= 1e-12
    assert n_inf > 5


def test_slsqp_cross_check():
    """An independent NLP solver reaches the same optimal cost."""
    b = gen.gen_cfg0(64)
    checked = 0
    for i in range(b.n):
        inst = b.instance(i)
        res = segment.solve(inst)
        if res.status != qp.SOLVED or abs(res.cost) < 1e-6:
            continue
        q = res.qp
        y0 = np.array(res.P.ravel()) + 1e-3
        sol = minimize(lambda y: y @ q.Q @ y, y0, jac=lambda y: 2 * q.Q @ y, method="SLSQP",
                       constraints=[{"type": "ineq", "fun": lambda y: q.u - q.A @ y, "jac": lambda y: -q.A},
                                    {"type": "eq", "fun": lambda y: q.E @ y - q.e, "jac": lambda y: q.E}],
                       options=dict(ftol=1e-15, maxiter=500))
        assert abs(sol.fun - res.cost) <= 1e-6 * abs(res.cost) + 1e-7
        checked += 1
        if checked >= 6:
            break
    assert checked >= 3


def test_cfg1_generator_infeasible_fraction():
    """About 30% of the cluttered-environment edges are infeasible."""
    b = gen.gen_cfg1(indices=range(300))
    st = np.array([segment.solve(b.instance(i)).status for i in range(b.n)])
    frac = np.mean(st == qp.INFEASIBLE)
    assert 0.2 <= frac <= 0.42
