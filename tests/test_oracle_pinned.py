"""Pins of the oracle's pinned-start-velocity variant (the full-state start of
Lemma 1: P_0 = pos(x0) and (p/T)(P_1 - P_0) = vel(x0)).

* With every inequality slack, the minimiser of int |b''|^2 under b(0) = x0,
  b'(0) = v0, b(T) = g is, by the calculus of variations, the cubic with the
  natural end condition b''(T) = 0 (the Euler-Lagrange equation b'''' = 0 and
  the free end derivative); every degree p >= 3 contains it, so the oracle
  must return it at any degree and duration, with its closed-form cost.
* A start speed above vmax in one coordinate is infeasible (the k = 0
  velocity row is a constant on the pinned set); below it, feasible.
* The pinned problem restricts the unpinned one: its optimum is feasible there
  and costs at least as much.
* Gradients through the pinned rows (envelope theorem and KKT adjoint) agree
  with central differences, including d/d vel(x0), which only the pin row
  carries."""
import numpy as np
import pytest

from oracle import qp, segment
from workloads import gen


def bernstein_curve(P, T, t):
    """Plain Bernstein sum b(t) = sum_k C(p,k) s^k (1-s)^(p-k) P_k, s = t/T."""
    from math import comb
    p = P.shape[0] - 1
    s = np.asarray(t)[:, None] / T
    return sum(comb(p, k) * s ** k * (1 - s) ** (p - k) * P[k] for k in range(p + 1))


def loose_instance(rng, p, T, pin=True):
    x0 = np.concatenate([rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)])
    g = x0[:3] + rng.uniform(-1, 1, 3)
    A = np.concatenate([np.eye(3), -np.eye(3)])
    b = np.full(6, 100.0)
    return dict(p=p, T=T, vmax=1e4, amax=1e6, A_face=A, b_face=b, H=np.zeros((0, 3 * (p + 1))),
                h0=np.zeros(0), G=np.zeros((0, 6)), x0=x0, goal=g, pin_v0=pin)


@pytest.mark.parametrize("p", [3, 5, 7, 9])
@pytest.mark.parametrize("T", [0.5, 1.0, 2.0])
def test_slack_pinned_optimum_is_the_natural_cubic(p, T):
    rng = np.random.default_rng(100 * p + int(10 * T))
    inst = loose_instance(rng, p, T)
    r = segment.solve(inst)
    assert r.status == qp.SOLVED and len(r.W) == 0
    x, v, g = inst["x0"][:3], inst["x0"][3:], inst["goal"]
    c3 = -(g - x - v * T) / (2 * T ** 3)
    c2 = -3 * c3 * T
    t = np.linspace(0, T, 101)
    want = x + v * t[:, None] + c2 * t[:, None] ** 2 + c3 * t[:, None] ** 3
    got = bernstein_curve(r.P, T, t)
    assert np.abs(got - want).max() <= 1e-9 * (1 + np.abs(want).max())
    a, bb = 2 * c2, 6 * c3
    f = a @ a * T + a @ bb * T ** 2 + bb @ bb * T ** 3 / 3
    assert abs(r.cost - f) <= 1e-9 * (1 + f)
    # the start derivative is the pinned velocity
    assert np.allclose(p / T * (r.P[1] - r.P[0]), v, rtol=0, atol=1e-12)


def test_unpinned_slack_optimum_is_a_line():
    """Control: without the pin the same instance relaxes to the straight
    segment (zero cost), so the pin is what bends the curve."""
    inst = loose_instance(np.random.default_rng(3), 7, 1.0, pin=False)
    r = segment.solve(inst)
    assert r.status == qp.SOLVED and r.cost <= 1e-20
    assert np.abs(np.diff(r.P, axis=0) - (inst["goal"] - inst["x0"][:3]) / 7).max() <= 1e-12


def test_start_speed_above_vmax_is_infeasible():
    inst = loose_instance(np.random.default_rng(4), 7, 1.0)
    inst["vmax"] = 3.0
    inst["x0"][3:] = [0.5, -3.5, 1.0]
    r = segment.solve(inst)
    assert r.status == qp.INFEASIBLE and r.certified
    inst["x0"][4] = -2.5
    assert segment.solve(inst).status == qp.SOLVED


def test_pinned_restricts_unpinned():
    b = gen.with_pinned_velocity(gen.gen_cfg1(indices=range(60)))
    n_cmp = 0
    for i in range(b.n):
        ip = b.instance(i)
        rp = segment.solve(ip)
        ru = segment.solve(dict(ip, pin_v0=False))
        if rp.status == qp.SOLVED:
            q = ru.qp
            y = rp.P.ravel()
            assert np.all(q.A @ y <= q.u + 1e-9 * (1 + np.abs(q.u)))
            assert np.abs(q.E @ y - q.e).max() <= 1e-9
            assert ru.status == qp.SOLVED and ru.cost <= rp.cost * (1 + 1e-9) + 1e-12
            n_cmp += 1
        if ru.status == qp.INFEASIBLE:
            assert rp.status == qp.INFEASIBLE
    assert n_cmp >= 10


def test_pinned_gradients_match_finite_differences():
    b = gen.with_pinned_velocity(gen.gen_cfg1(indices=range(80)))
    rng = np.random.default_rng(12)
    done = 0
    for i in range(b.n):
        inst = b.instance(i)
        res = segment.solve(inst)
        if not (res.status == qp.SOLVED and segment.gradient_certified(res) and len(res.W) > 0):
            continue
        gbar = rng.standard_normal(res.P.size)
        gx0, ggoal, gb = segment.gradients(res, gbar).combined(0.7)
        fd = segment.fd_gradients(inst, gbar, 0.7, h=1e-6)
        for got, want in ((gx0, fd["x0"]), (ggoal, fd["goal"]), (gb, fd["b"])):
            assert np.linalg.norm(got - want) <= 1e-5 * max(np.linalg.norm(want), 1.0), (i, got, want)
        # the pin row is what carries d/d vel(x0)
        assert np.linalg.norm(gx0[3:]) > 1e-6
        done += 1
        if done >= 4:
            break
    assert done >= 3
