"""Pins of the MPC refinement oracle (eq. MPC, Sec. III-D) against results
that do not go through its own assembly:

* a reference that the dynamics can follow exactly, with no input or length
  cost, is tracked exactly (zero cost, the generating inputs);
* with every inequality slack the optimum equals the equality-constrained
  least-squares solution in the inputs alone, states eliminated by rolling
  the motion p(t) = p + v t + u t^2 / 2 forward (a different formulation of
  the same problem);
* a two-step horizon has exactly one feasible point, found by a 6 x 6 solve;
* the control points used for the keep-out rows reproduce the motion over
  the step (Lemma 1), so the plane rows keep the sampled motion on the free
  side (Property 1);
* optima of generated instances satisfy the dynamics, every row and the KKT
  conditions, and dropping the planes never raises the cost; a plane that
  cuts the fixed start is certified infeasible."""
from math import comb

import numpy as np
import pytest

from oracle import mpc, qp
from workloads import gen


def step(x, u, dt):
    """Motion under a constant acceleration for one step."""
    p, v = x[:3], x[3:]
    return np.concatenate([p + dt * v + 0.5 * dt * dt * u, v + dt * u])


def rollout(x0, U, dt):
    X = [np.asarray(x0, float)]
    for u in U:
        X.append(step(X[-1], u, dt))
    return np.array(X)


def loose(b, i):
    inst = b.instance(i)
    inst["planes"] = inst["planes"].copy()
    inst["planes"][:, 3] = -1e3          # n . y >= -1000: never active
    inst["G"] = np.full_like(inst["G"], 1e3)
    return inst


def test_feasible_reference_is_tracked_exactly():
    b = gen.gen_mpc(4, N=20)
    rng = np.random.default_rng(1)
    for i in range(b.n):
        inst = loose(b, i)
        U = rng.uniform(-0.5, 0.5, (inst["N"], 3))
        inst["ref"] = rollout(inst["x0"], U, inst["dt"])
        inst["R"] = np.zeros((3, 3))
        inst["w"] = 0.0
        r = mpc.solve(inst)
        assert r.status == qp.SOLVED
        assert np.abs(r.X - inst["ref"]).max() <= 1e-9
        assert np.abs(r.U - U).max() <= 1e-7
        assert abs(r.cost) <= 1e-12


def test_slack_optimum_equals_condensed_least_squares():
    b = gen.gen_mpc(3, N=25)
    for i in range(b.n):
        inst = loose(b, i)
        N, dt = inst["N"], inst["dt"]
        Q, R, w = inst["Q"], inst["R"], inst["w"]
        x0, ref = inst["x0"], inst["ref"]
        base = rollout(x0, np.zeros((N, 3)), dt)
        cols = []
        for j in range(3 * N):
            Uj = np.zeros(3 * N); Uj[j] = 1.0
            cols.append(rollout(np.zeros(6), Uj.reshape(N, 3), dt) - rollout(np.zeros(6), np.zeros((N, 3)), dt))
        cols = np.array(cols)                            # [3N, N+1, 6]: state response to unit inputs
        sq, sr = np.sqrt(np.diag(Q)), np.linalg.cholesky(R).T
        rows, rhs = [], []
        for k in range(1, N):                            # tracking
            rows.append(sq[:, None] * cols[:, k, :].T); rhs.append(sq * (ref[k] - base[k]))
        for k in range(N):                               # inputs
            Rk = np.zeros((3, 3 * N)); Rk[:, 3 * k:3 * k + 3] = sr
            rows.append(Rk); rhs.append(np.zeros(3))
        for k in range(N):                               # squared step length
            d = cols[:, k + 1, :3] - cols[:, k, :3]
            rows.append(np.sqrt(w) * d.T); rhs.append(-np.sqrt(w) * (base[k + 1, :3] - base[k, :3]))
        L, t = np.vstack(rows), np.concatenate(rhs)
        C = cols[:, N, :].T                              # terminal state
        K = np.block([[2 * L.T @ L, C.T], [C, np.zeros((6, 6))]])
        sol = np.linalg.solve(K, np.concatenate([2 * L.T @ t, ref[N] - base[N]]))
        u = sol[:3 * N]
        want_cost = float(np.sum((L @ u - t) ** 2))
        r = mpc.solve(inst)
        assert r.status == qp.SOLVED and not r.W
        assert np.abs(r.U.ravel() - u).max() <= 1e-8 * (1 + np.abs(u).max())
        assert abs(r.cost - want_cost) <= 1e-9 * (1 + want_cost)


def test_two_step_horizon_has_one_point():
    b = gen.gen_mpc(3, N=2)
    for i in range(b.n):
        inst = loose(b, i)
        x0, dt, rN = inst["x0"], inst["dt"], inst["ref"][2]
        # r_N = step(step(x0, u0), u1) is linear in (u0, u1)
        z = rollout(x0, np.zeros((2, 3)), dt)[2]
        M = np.zeros((6, 6))
        for j in range(6):
            e = np.zeros(6); e[j] = 1.0
            M[:, j] = rollout(np.zeros(6), e.reshape(2, 3), dt)[2]
        u = np.linalg.solve(M, rN - z)
        r = mpc.solve(inst)
        assert r.status == qp.SOLVED
        assert np.abs(r.U.ravel() - u).max() <= 1e-8 * (1 + np.abs(u).max())
        assert np.abs(r.X - rollout(x0, u.reshape(2, 3), dt)).max() <= 1e-9


def test_cubic_points_reproduce_the_step():
    rng = np.random.default_rng(2)
    for _ in range(20):
        x, u, dt = rng.standard_normal(6), rng.standard_normal(3), rng.uniform(0.05, 0.5)
        x1 = step(x, u, dt)
        P = mpc.cubic_points(x, x1, dt)
        for t in np.linspace(0.0, dt, 11):
            s = t / dt
            b = sum(comb(3, k) * s ** k * (1 - s) ** (3 - k) * P[k] for k in range(4))
            assert np.abs(b - (x[:3] + t * x[3:] + 0.5 * t * t * u)).max() <= 1e-12


@pytest.fixture(scope="module")
def solved():
    b = gen.gen_mpc(6)
    return b, [mpc.solve(b.instance(i)) for i in range(b.n)]


def test_generated_optima_are_feasible_and_stationary(solved):
    b, res = solved
    n_active = 0
    for i, r in enumerate(res):
        assert r.status == qp.SOLVED and r.kkt["max"] <= 1e-9
        inst = b.instance(i)
        dt = inst["dt"]
        assert np.abs(r.X[0] - inst["x0"]).max() == 0 or np.abs(r.X[0] - inst["x0"]).max() <= 1e-12
        assert np.abs(r.X[-1] - inst["ref"][-1]).max() <= 1e-10
        for k in range(inst["N"]):
            assert np.abs(r.X[k + 1] - step(r.X[k], r.U[k], dt)).max() <= 1e-10
            assert np.all(inst["F1"] @ r.X[k] + inst["F2"] @ r.X[k + 1] <= inst["G"] + 1e-9)
            n, l = inst["planes"][k, :3], inst["planes"][k, 3]
            for t in np.linspace(0.0, dt, 21):
                p = r.X[k, :3] + t * r.X[k, 3:] + 0.5 * t * t * r.U[k]
                assert n @ p >= l - 1e-9
        n_active += len(r.W)
    assert n_active >= 6


def test_dropping_planes_never_raises_the_cost(solved):
    b, res = solved
    for i, r in enumerate(res):
        inst = b.instance(i)
        inst["planes"] = inst["planes"].copy()
        inst["planes"][:, 3] = -1e3
        r2 = mpc.solve(inst)
        assert r2.status == qp.SOLVED and r2.cost <= r.cost * (1 + 1e-10) + 1e-12


def test_plane_through_the_start_is_infeasible():
    b = gen.gen_mpc(1)
    inst = b.instance(0)
    inst["planes"] = inst["planes"].copy()
    n = inst["planes"][0, :3]
    inst["planes"][0, 3] = n @ inst["x0"][:3] + 0.05     # the fixed start is 0.05 on the wrong side
    r = mpc.solve(inst)
    assert r.status == qp.INFEASIBLE and r.s_star >= qp.TAU


def _old_scalar_bound(inst):
    """The earlier |y|_inf bound, which read max(G) as the velocity limit and
    max(G)/dt as the input limit: valid for the generated box rows only."""
    G, dt, N = np.asarray(inst["G"]), float(inst["dt"]), int(inst["N"])
    vmax = max(float(np.max(G)), float(np.max(np.abs(inst["x0"][3:]))))
    return float(np.max(np.abs(inst["x0"][:3])) + (N + 1) * dt * vmax + vmax + float(np.max(G)) / dt + 2.0)


def _skewed_rows(dt):
    """Reachable rows that are not a velocity box and an input box: two
    nearly parallel pairs of velocity rows (|v_x - 0.98 v_y| and
    |v_x - 0.99 v_y| at most 0.05 after normalisation), which leave v_y free
    up to about 10 m/s although every right-hand side is small, a box on
    v_z, and an input box |v_{k+1} - v_k| <= 0.4."""
    r1, r2, g = [], [], []
    for a, gg in (((1.0, -0.98, 0.0), 0.05), ((1.0, -0.99, 0.0), 0.05), ((0.0, 0.0, 1.0), 0.05)):
        a = np.asarray(a) / np.linalg.norm(a)
        for sgn in (1.0, -1.0):
            z = np.zeros(6); w = np.zeros(6); w[3:] = sgn * a
            r1.append(z); r2.append(w); g.append(gg)
    for c in range(3):
        for sgn in (1.0, -1.0):
            z = np.zeros(6); w = np.zeros(6); z[3 + c] = -sgn; w[3 + c] = sgn
            r1.append(z); r2.append(w); g.append(0.4)
    return np.array(r1), np.array(r2), np.array(g)


def _skewed_instance(N=40, dt=0.1):
    F1, F2, G = _skewed_rows(dt)
    return dict(N=N, dt=dt, Q=np.diag([1.0, 1, 1, 0.1, 0.1, 0.1]), R=0.01 * np.eye(3), w=1.0,
                F1=F1, F2=F2, G=G, x0=np.zeros(6), ref=np.zeros((N + 1, 6)),
                planes=np.tile(np.array([0.0, 0.0, 1.0, -1e3]), (N, 1)))


def _exact_extreme(inst, idx, sgn):
    """max of sgn * y[idx] over x_0 = x0, the dynamics and the reachable rows
    (the relaxation the box encloses), by one LP over the whole horizon."""
    from scipy.optimize import linprog
    q = mpc.build(inst)
    N = inst["N"]
    m = len(inst["G"])
    A = q.A[:N * m]                     # reachable rows come first
    u = q.u[:N * m]
    E, e = q.E, q.e
    keep = np.r_[0:6 + 6 * N, E.shape[0] - 1]           # drop the terminal state
    c = np.zeros(q.A.shape[1]); c[idx] = -sgn
    res = linprog(c, A_ub=A, b_ub=u, A_eq=E[keep], b_eq=e[keep], bounds=[(None, None)] * len(c),
                  method="highs")
    assert res.status == 0
    return -float(res.fun)


def test_feasible_box_encloses_the_exact_extremes_of_skewed_rows():
    """The box from the instance's own rows contains the exact LP extremes
    of positions, velocities and inputs on rows that are not boxes, while the
    earlier max(G) reading falls short of them (so it could have certified a
    feasible instance as infeasible)."""
    inst = _skewed_instance()
    lo, hi = mpc.feasible_box(inst)
    N = inst["N"]
    iy_p = 6 * N + 1           # p_y at the last node
    iy_v = 6 * (N // 2) + 4    # v_y half way
    iu = 6 * (N + 1) + 3 * (N // 2) + 1
    for idx in (iy_p, iy_v, iu, 6 * N):
        top, bot = _exact_extreme(inst, idx, 1.0), -_exact_extreme(inst, idx, -1.0)
        assert lo[idx] <= bot + 1e-9 and top <= hi[idx] + 1e-9, (idx, lo[idx], bot, top, hi[idx])
    assert _exact_extreme(inst, iy_p, 1.0) > 1.2 * _old_scalar_bound(inst)


def test_feasible_box_encloses_generated_optima(solved):
    b, res = solved
    for i, r in enumerate(res):
        lo, hi = mpc.feasible_box(b.instance(i))
        assert np.all(r.y >= lo - 1e-9) and np.all(r.y <= hi + 1e-9)


def test_plane_through_the_start_is_infeasible_with_skewed_rows():
    inst = _skewed_instance(N=12)
    inst["planes"] = inst["planes"].copy()
    inst["planes"][0] = [1.0, 0.0, 0.0, 0.05]      # the fixed start (origin) is 0.05 on the wrong side
    r = mpc.solve(inst)
    assert r.status == qp.INFEASIBLE and r.s_star >= qp.TAU


def test_unbounded_rows_are_never_certified():
    """Rows that leave the relaxed set unbounded give no box, and the
    phase-1 check then certifies nothing (the class stays uncertified)."""
    inst = _skewed_instance(N=6)
    keep = [0, 1, 2, 3]                                # only the skewed velocity pairs: v_z and inputs free
    inst["F1"], inst["F2"], inst["G"] = inst["F1"][keep], inst["F2"][keep], inst["G"][keep]
    assert mpc.feasible_box(inst) is None
    inst["planes"] = inst["planes"].copy()
    inst["planes"][0] = [1.0, 0.0, 0.0, 0.05]
    r = mpc.solve(inst)
    assert r.status == qp.UNCERTIFIED
