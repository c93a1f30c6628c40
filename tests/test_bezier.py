"""Pins of the oracle's Bezier mathematics (Sec. II-B, Properties 1-3).

Each check compares against something computed another way: numpy's power
basis polynomial arithmetic, quadrature, or a textbook closed form."""
import numpy as np
import pytest
from math import comb
from numpy.polynomial import polynomial as npoly
from numpy.polynomial.legendre import leggauss

from oracle import bezier


def power_basis(P, T):
    """Each coordinate of the curve as a power-series polynomial in t,
    expanded from C(p,i) (t/T)^i (1 - t/T)^(p-i) with numpy's polynomial
    arithmetic (independent of the Bernstein code under test)."""
    p = P.shape[0] - 1
    polys = []
    for c in range(P.shape[1]):
        acc = np.zeros(1)
        for i in range(p + 1):
            s = np.array([0.0, 1.0 / T])
            one_minus = np.array([1.0, -1.0 / T])
            term = comb(p, i) * npoly.polymul(npoly.polypow(s, i), npoly.polypow(one_minus, p - i))
            acc = npoly.polyadd(acc, P[i, c] * term)
        polys.append(acc)
    return polys


@pytest.mark.parametrize("p", range(1, 10))
def test_bernstein_matches_decasteljau(p):
    rng = np.random.default_rng(p)
    P = rng.uniform(-10, 10, size=(p + 1, 3))
    s = np.linspace(0, 1, 101)
    closed = bezier.bernstein(p, s) @ P
    dc = np.array([bezier.decasteljau(P, si) for si in s])
    assert np.max(np.abs(closed - dc)) <= 1e-13 * (1 + np.abs(P).max())


@pytest.mark.parametrize("p", range(1, 10))
def test_partition_of_unity_and_endpoints(p):
    B = bezier.bernstein(p, np.linspace(0, 1, 57))
    assert np.allclose(B.sum(1), 1.0, atol=1e-14)
    rng = np.random.default_rng(10 + p)
    P = rng.standard_normal((p + 1, 3))
    T = 0.7
    assert np.allclose(bezier.curve_bernstein(P, 0.0, T), P[0], atol=1e-14)
    assert np.allclose(bezier.curve_bernstein(P, T, T), P[-1], atol=1e-13)


@pytest.mark.parametrize("p,T", [(3, 1.0), (5, 0.5), (7, 1.0), (9, 2.0)])
@pytest.mark.parametrize("order", [1, 2])
def test_derivative_points_match_polynomial_derivative(p, T, order):
    """The derivative map of Sec. II-B: the order-k derivative is a Bezier
    curve whose control points are p!/(p-k)!/T^k Delta^k P."""
    rng = np.random.default_rng(100 * p + order)
    P = rng.uniform(-5, 5, size=(p + 1, 3))
    D = bezier.derivative_points(P, order, T)
    t = np.linspace(0, T, 33)
    got = bezier.curve_bernstein(D, t, T)
    want = np.stack([npoly.polyval(t, npoly.polyder(c, order)) for c in power_basis(P, T)], axis=1)
    assert np.max(np.abs(got - want)) <= 1e-9 * (1 + np.abs(want).max())


@pytest.mark.parametrize("n", range(0, 8))
def test_bernstein_gram_is_the_l2_gram(n):
    x, w = leggauss(n + 2)
    s = (x + 1) / 2
    B = bezier.bernstein(n, s)
    M = (B * (w / 2)[:, None]).T @ B
    assert np.max(np.abs(M - bezier.bernstein_gram(n))) <= 1e-14


@pytest.mark.parametrize("p", range(3, 10))
@pytest.mark.parametrize("T", [0.5, 1.0, 2.0])
def test_hessian_is_the_integrated_squared_second_derivative(p, T):
    """y^T Q y equals int_0^T |b''|^2, integrated exactly from numpy's
    power-basis second derivative (the segment cost)."""
    rng = np.random.default_rng(7 * p)
    Q = bezier.hessian(p, T)
    for _ in range(3):
        P = rng.uniform(-3, 3, size=(p + 1, 3))
        want = 0.0
        for c in power_basis(P, T):
            d2 = npoly.polyder(c, 2)
            sq = npoly.polyint(npoly.polymul(d2, d2))
            want += npoly.polyval(T, sq) - npoly.polyval(0.0, sq)
        got = P.ravel() @ Q @ P.ravel()
        # the power basis loses ~7 digits at p = 9, T = 0.5 to cancellation
        assert abs(got - want) <= 1e-8 * (1 + abs(want))


def test_cubic_cost_closed_form():
    """A cubic's second derivative is linear with end values 6 a / T^2 and
    6 c / T^2 (a = Delta^2 P_0, c = Delta^2 P_1), so
    f = (36 / T^3) (|a|^2 + a.c + |c|^2) / 3."""
    rng = np.random.default_rng(3)
    for T in (0.5, 1.0, 3.0):
        P = rng.standard_normal((4, 3))
        a = P[2] - 2 * P[1] + P[0]
        c = P[3] - 2 * P[2] + P[1]
        want = 36.0 / T ** 3 * (a @ a + a @ c + c @ c) / 3.0
        got = P.ravel() @ bezier.hessian(3, T) @ P.ravel()
        assert abs(got - want) <= 1e-12 * (1 + want)


@pytest.mark.parametrize("p", range(3, 10))
def test_hessian_null_space_is_affine_sequences(p):
    """Only straight lines traversed at constant speed cost nothing: the
    null space of Q_1D is spanned by the constant and linear sequences."""
    Q1 = bezier.hessian_1d(p, 1.0)
    k = np.arange(p + 1, dtype=float)
    assert np.allclose(Q1 @ np.ones(p + 1), 0, atol=1e-9)
    assert np.allclose(Q1 @ k, 0, atol=1e-9)
    ev = np.linalg.eigvalsh(Q1)
    assert np.sum(ev < 1e-8 * ev.max()) == 2
    # interior block (both end points pinned) is positive definite
    assert np.linalg.eigvalsh(Q1[1:p, 1:p]).min() > 0


def test_convex_hull_property():
    """Property 1: every curve point is a convex combination of the control
    points, so it satisfies every halfspace the control points satisfy."""
    rng = np.random.default_rng(5)
    for p in (3, 7, 9):
        A = rng.standard_normal((12, 3))
        P = rng.uniform(-1, 1, size=(p + 1, 3))
        b = (P @ A.T).max(0)
        pts = bezier.curve_bernstein(P, np.linspace(0, 1, 1001))
        assert np.all(pts @ A.T <= b + 1e-12)


def test_subdivision_reproduces_the_curve():
    """Property 3: the two halves of a split reproduce the curve."""
    rng = np.random.default_rng(6)
    P = rng.standard_normal((8, 3))
    s0 = 0.37
    left, right = bezier.split(P, s0)
    u = np.linspace(0, 1, 21)
    assert np.allclose(bezier.curve_bernstein(left, u), bezier.curve_bernstein(P, u * s0), atol=1e-13)
    assert np.allclose(bezier.curve_bernstein(right, u), bezier.curve_bernstein(P, s0 + u * (1 - s0)), atol=1e-13)


def test_path_length_bound():
    """Property 2: the control-polygon length bounds the arc length."""
    rng = np.random.default_rng(8)
    for _ in range(5):
        P = rng.standard_normal((8, 3))
        t = np.linspace(0, 1, 20001)
        pts = bezier.curve_bernstein(P, t)
        arc = np.linalg.norm(np.diff(pts, axis=0), axis=1).sum()
        assert arc <= bezier.path_length_bound(P) + 1e-9
