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
