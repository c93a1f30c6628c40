"""Pins of the oracle's derivatives of the optimum.

Three routes must agree on instances whose active set is stable under small
perturbations (non-degenerate multipliers, inactive rows with slack):
the envelope theorem for the optimal cost, the KKT adjoint for any linear
functional of P*, and central finite differences of re-solved problems."""
import numpy as np
import pytest

from oracle import qp, segment
from workloads import gen


def certified(b, limit):
    out = []
    for i in range(b.n):
        inst = b.instance(i)
        res = segment.solve(inst)
        if res.status == qp.SOLVED and segment.gradient_certified(res) and len(res.W) > 0:
            out.append((inst, res))
        if len(out) >= limit:
            break
    return out


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-8)


@pytest.fixture(scope="module")
def cases():
    return certified(gen.gen_cfg0(64), 4) + certified(gen.gen_cfg1(indices=range(40)), 4)


def test_have_cases(cases):
    assert len(cases) >= 6


def test_envelope_equals_chain_rule_through_adjoint(cases):
    """df*/dtheta = (2 Q y*)^T dy*/dtheta: the adjoint VJP with upstream
    2 Q y* must reproduce the envelope-theorem gradient."""
    for inst, res in cases:
        g = segment.gradients(res)
        chain = segment.gradients(res, 2.0 * res.qp.Q @ res.P.ravel())
        assert rel(chain.sol_x0, g.cost_x0) <= 1e-8
        assert rel(chain.sol_goal, g.cost_goal) <= 1e-8
        assert rel(chain.sol_b, g.cost_b) <= 1e-8 or np.linalg.norm(g.cost_b) < 1e-8


def test_gradients_match_central_differences(cases):
    rng = np.random.default_rng(4)
    for inst, res in cases[:5]:
        gbar = rng.standard_normal(res.P.size)
        gx0, ggoal, gb = segment.gradients(res, gbar).combined(1.0)
        fd = segment.fd_gradients(inst, gbar, 1.0, h=1e-6)
        assert rel(gx0, fd["x0"]) <= 1e-4
        assert rel(ggoal, fd["goal"]) <= 1e-4
        assert rel(gb, fd["b"]) <= 1e-4 or np.linalg.norm(fd["b"]) < 1e-6


def test_unconstrained_goal_gradient_closed_form():
    """With no active inequality the optimum is the straight line, f* = 0 and
    P*_k = P_0 + (k/p)(goal - P_0): dP*_k/dgoal = k/p, dP*_k/dP_0 = 1 - k/p."""
    from tests.test_oracle_qp import line_instance
    inst = line_instance(p=7, seed=2)
    res = segment.solve(inst)
    assert len(res.W) == 0
    p = inst["p"]
    rng = np.random.default_rng(1)
    gbar = rng.standard_normal((p + 1, 3))
    g = segment.gradients(res, gbar.ravel())
    k = np.arange(p + 1)[:, None] / p
    assert np.allclose(g.sol_goal, (gbar * k).sum(0), atol=1e-10)
    assert np.allclose(g.sol_x0[:3], (gbar * (1 - k)).sum(0), atol=1e-10)
    assert np.allclose(g.sol_x0[3:], 0.0)
    assert np.allclose(g.cost_x0, 0.0, atol=1e-9) and np.allclose(g.cost_goal, 0.0, atol=1e-9)
