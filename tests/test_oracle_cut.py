"""Pins of the Cut-QP / cut-heuristic oracle (Sec. III-B, Alg. 2, eq. Cut-QP)
against facts that do not come from the oracle itself: closed-form
point-to-box and segment-to-box distances, brute force over sampled convex
combinations, a separating-plane lower bound that must equal the returned
distance, the LP feasibility of conv(P) meeting the box, the Cut-QP objective
evaluated at the returned point, and geometric invariances."""
import numpy as np
import pytest

from oracle import cut
from workloads import gen


def rand_box(rng):
    c = rng.uniform(-2, 2, 3)
    w = rng.uniform(0.2, 1.5, 3)
    return c - w / 2, c + w / 2


def test_single_point_is_point_to_box_distance():
    rng = np.random.default_rng(1)
    for _ in range(200):
        lo, hi = rand_box(rng)
        x = rng.uniform(-4, 4, 3)
        P = np.tile(x, (8, 1))
        want = float(np.sum((x - np.clip(x, lo, hi)) ** 2))
        assert abs(cut.cut_qp(P, lo, hi).dist2 - want) <= 1e-12 * (1 + want)


def test_axis_parallel_segment_closed_form():
    """Segment from (a, y, z) to (b, y, z): the distance along x is the gap
    between [a, b] and [lo_x, hi_x]; y and z add their own gaps."""
    rng = np.random.default_rng(2)
    for _ in range(200):
        lo, hi = rand_box(rng)
        a, b = np.sort(rng.uniform(-4, 4, 2))
        y, z = rng.uniform(-4, 4, 2)
        P = np.array([[a + (b - a) * k / 3, y, z] for k in range(4)])
        gx = max(0.0, lo[0] - b, a - hi[0])
        gy = max(0.0, lo[1] - y, y - hi[1])
        gz = max(0.0, lo[2] - z, z - hi[2])
        want = gx * gx + gy * gy + gz * gz
        assert abs(cut.cut_qp(P, lo, hi).dist2 - want) <= 1e-11 * (1 + want)


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_and_separating_plane_bound(seed):
    """Upper bound: no sampled point of conv(P) is closer to the box than the
    optimum.  Lower bound: the plane with normal n = x* - y* separates the
    control points from the box by exactly |n|, so the distance is pinned
    from both sides."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(20):
        lo, hi = rand_box(rng)
        P = rng.uniform(-3, 3, (8, 3))
        r = cut.cut_qp(P, lo, hi)
        lam = rng.dirichlet(np.ones(8) * 0.3, size=4000)
        X = lam @ P
        sampled = np.min(np.sum((X - np.clip(X, lo, hi)) ** 2, axis=1))
        assert r.dist2 <= sampled + 1e-12
        if r.dist2 > 1e-12:
            n = r.x - r.y
            corners = cut.box_corners(lo, hi)
            gap = np.min(P @ n) - np.max(corners @ n)
            assert gap >= r.dist2 * (1 - 1e-9) - 1e-12
            assert abs(np.linalg.norm(n) ** 2 - r.dist2) <= 1e-10 * (1 + r.dist2)


def test_cut_qp_objective_at_the_returned_point():
    """The returned (lam, delta) is feasible for the Cut-QP as written and its
    objective |delta|^2 equals the optimum (delta = (A P^T lam - b)_+).  The
    weights come from an LP solve, so they hold to its feasibility tolerance
    (about 1e-7); the optimum itself is the exact hull distance."""
    rng = np.random.default_rng(3)
    for _ in range(100):
        lo, hi = rand_box(rng)
        P = rng.uniform(-3, 3, (8, 3))
        r = cut.cut_qp(P, lo, hi)
        A, b = cut.box_rows(lo, hi)
        assert np.all(r.lam >= -1e-9) and abs(r.lam.sum() - 1) <= 1e-7
        assert np.all(A @ (P.T @ r.lam) <= b + r.delta + 1e-7)
        assert abs(float(r.delta @ r.delta) - r.dist2) <= 1e-6 * (1 + r.dist2)


def test_zero_exactly_when_the_lp_finds_a_common_point():
    rng = np.random.default_rng(4)
    n_meet = 0
    for _ in range(300):
        lo, hi = rand_box(rng)
        P = rng.uniform(-2.5, 2.5, (8, 3))
        s = cut.lp_margin(P, lo, hi)
        if abs(s) < cut.TAU:
            continue
        d2 = cut.cut_qp(P, lo, hi).dist2
        assert (d2 == 0.0) == (s < 0), (s, d2)
        n_meet += s < 0
    assert 20 < n_meet < 280


def test_translation_and_reflection_invariance():
    rng = np.random.default_rng(5)
    for _ in range(50):
        lo, hi = rand_box(rng)
        P = rng.uniform(-3, 3, (8, 3))
        d = cut.cut_qp(P, lo, hi).dist2
        t = rng.uniform(-5, 5, 3)
        assert abs(cut.cut_qp(P + t, lo + t, hi + t).dist2 - d) <= 1e-9 * (1 + d)
        f = np.array([-1.0, 1.0, 1.0])
        assert abs(cut.cut_qp(P * f, np.minimum(lo * f, hi * f), np.maximum(lo * f, hi * f)).dist2 - d) <= 1e-9 * (1 + d)


def test_heuristic_steps_agree_with_the_exact_answer():
    """Each step of Alg. 2 is a certificate: step 1 finds a common point,
    step 2 a plane that keeps every box corner on the near side and every
    control point strictly on the far side; all steps match the Cut-QP."""
    b = gen.gen_cut(n_nodes=300, k_nn=6, n_obst=60)
    rng = np.random.default_rng(6)
    seen = set()
    for e in rng.choice(b.n_edges, 40, replace=False):
        for o in range(b.n_obstacles):
            P, lo, hi = b.P[e], b.box_lo[o], b.box_hi[o]
            code, step, d2 = cut.heuristic(P, lo, hi)
            seen.add(step)
            if step == cut.BY_POINT:
                assert code == cut.CUT
                assert np.any(np.all((P >= lo) & (P <= hi), axis=1))
            elif step == cut.BY_PLANE:
                assert code == cut.FREE
                n, l = cut.adjacent_hyperplane(P, lo, hi, cut.closest_point(P, lo, hi))
                assert np.all(cut.box_corners(lo, hi) @ n <= l + 1e-12) and np.all(P @ n > l)
            # the LP certificate on a sample of the pairs (one LP each)
            if step != cut.BY_QP and (step == cut.BY_POINT or rng.random() < 0.05) \
                    and abs(cut.lp_margin(P, lo, hi)) >= cut.TAU:
                assert (cut.cut_qp(P, lo, hi).dist2 > 0) == (code == cut.FREE)
    assert cut.BY_PLANE in seen


def test_workload_shape():
    b = gen.gen_cut(n_nodes=500, k_nn=10, n_obst=50)
    assert b.P.shape == (5000, 8, 3) and b.box_lo.shape == (50, 3)
    assert np.all(b.box_hi > b.box_lo)
    b2 = gen.gen_cut(n_nodes=500, k_nn=10, n_obst=50)
    assert np.array_equal(b.P, b2.P)


# ---------------------------------------------------------------------------
# Polytope obstacles {x : A x <= b}
# ---------------------------------------------------------------------------
def rand_polytope(rng, k=None):
    off, A, b = gen.polytope_obstacles(1, rng, extent=2.0)
    return A, b


def test_box_as_polytope_is_the_squared_distance():
    """With the box's six unit rows the Cut-QP optimum is the squared
    Euclidean distance between conv(P) and the box (computed independently
    by the hull-projection routine)."""
    rng = np.random.default_rng(21)
    for _ in range(60):
        lo, hi = rand_box(rng)
        P = rng.uniform(-3, 3, (8, 3)) * rng.uniform(0.1, 1.0) + rng.uniform(-3, 3, 3)
        A, b = cut.box_rows(lo, hi)
        want = cut.cut_qp(P, lo, hi).dist2
        got = cut.cut_qp_poly(P, A, b)
        assert abs(got.value - want) <= 1e-12 * (1 + want), (got.value, want)


def test_single_point_closed_form():
    """All control points equal to x: the only convex combination is x, and
    the optimum is |(A x - b)_+|^2."""
    rng = np.random.default_rng(22)
    for _ in range(100):
        A, b = rand_polytope(rng)
        x = rng.uniform(-2, 4, 3)
        want = float(np.sum(np.maximum(A @ x - b, 0.0) ** 2))
        assert abs(cut.cut_qp_poly(np.tile(x, (8, 1)), A, b).value - want) <= 1e-12 * (1 + want)


@pytest.mark.parametrize("seed", range(4))
def test_polytope_value_enclosed_by_duality_and_sampling(seed):
    """Weak duality: the dual value h(2 delta) <= optimum <= f(lam) at the
    returned weights, and the two meet; every sampled convex combination has
    f >= the optimum."""
    rng = np.random.default_rng(300 + seed)
    for _ in range(15):
        A, b = rand_polytope(rng)
        P = rng.uniform(-2, 2, (8, 3)) * rng.uniform(0.2, 1.0) + rng.uniform(-2, 4, 3)
        r = cut.cut_qp_poly(P, A, b)
        assert r.lower <= r.value + 1e-13 * (1 + r.value)
        assert r.value - r.lower <= 1e-10 * (1 + r.value), (r.value, r.lower)
        assert abs(r.lam.sum() - 1.0) <= 1e-14 and np.all(r.lam >= 0)
        M = A @ P.T
        lam = rng.dirichlet(np.ones(8) * 0.3, size=3000)
        F = np.sum(np.maximum(lam @ M.T - b, 0.0) ** 2, axis=1)
        assert r.value <= F.min() + 1e-12
        # any mu >= 0 is a lower bound
        for _ in range(20):
            mu = rng.exponential(1.0, A.shape[0]) * rng.uniform(0, 3)
            assert cut.poly_dual(M, b, mu) <= r.value + 1e-12


def test_polytope_zero_exactly_when_the_lp_finds_a_common_point():
    rng = np.random.default_rng(23)
    n_zero = n_pos = 0
    for _ in range(150):
        A, b = rand_polytope(rng)
        P = rng.uniform(-1.5, 1.5, (8, 3)) * rng.uniform(0.2, 1.0) + rng.uniform(-1, 3, 3)
        s = cut.poly_lp_margin(P, A, b)
        if abs(s) < cut.TAU:
            continue
        v = cut.cut_qp_poly(P, A, b).value
        if s < 0:
            assert v == 0.0
            n_zero += 1
        else:
            assert v > 0.0
            n_pos += 1
    assert n_zero > 10 and n_pos > 10


def test_polytope_scaling_and_translation():
    """Scaling every row and offset by s scales the optimum by s^2;
    translating the control points by t and the offsets by A t leaves it."""
    rng = np.random.default_rng(24)
    for _ in range(30):
        A, b = rand_polytope(rng)
        P = rng.uniform(-2, 2, (8, 3)) * 0.5 + rng.uniform(-2, 4, 3)
        v = cut.cut_qp_poly(P, A, b).value
        s = rng.uniform(0.3, 3.0)
        assert abs(cut.cut_qp_poly(P, s * A, s * b).value - s * s * v) <= 1e-11 * (1 + s * s * v)
        t = rng.uniform(-5, 5, 3)
        assert abs(cut.cut_qp_poly(P + t, A, b + A @ t).value - v) <= 1e-11 * (1 + v)


def test_polytope_closest_point_kkt():
    """The closest point of O to the centroid: inside O a point is its own
    projection; outside, c - x* is a non-negative combination of the rows
    tight at x* (checked by non-negative least squares)."""
    from scipy.optimize import nnls
    rng = np.random.default_rng(25)
    for _ in range(60):
        A, b = rand_polytope(rng)
        P = rng.uniform(-2, 2, (8, 3)) * 0.3 + rng.uniform(-2, 4, 3)
        c = P.mean(axis=0)
        x = cut.poly_closest_point(P, A, b)
        assert np.all(A @ x <= b + 1e-10)
        if np.all(A @ c <= b):
            assert np.abs(x - c).max() <= 1e-12
            continue
        tight = np.nonzero(A @ x >= b - 1e-9)[0]
        mu, res = nnls(A[tight].T, c - x)
        assert res <= 1e-9 * (1 + np.abs(c - x).max())


def test_polytope_heuristic_steps_are_certificates():
    """Step 1: a control point inside O (so v* = 0); step 2: the plane keeps
    O on its near side (LP support) and every control point beyond it (so
    v* > 0); step 3 agrees with the LP decision on certified margins."""
    b = gen.gen_cut(n_nodes=200, k_nn=5, n_obst=0, n_poly=25)
    rng = np.random.default_rng(26)
    seen = set()
    for e in rng.choice(b.n_edges, 25, replace=False):
        for j in range(b.n_polytopes):
            A, bb = b.polytope(j)
            P = b.P[e]
            code, step, v = cut.heuristic_poly(P, A, bb)
            seen.add(step)
            if step == cut.BY_POINT:
                assert code == cut.CUT and np.any(np.all(P @ A.T <= bb, axis=1))
            elif step == cut.BY_PLANE:
                n = P.mean(axis=0) - cut.poly_closest_point(P, A, bb)
                l = cut.poly_support(A, bb, n)
                assert code == cut.FREE and np.all(P @ n > l)
            else:
                s = cut.poly_lp_margin(P, A, bb)
                if abs(s) >= cut.TAU:
                    assert (code == cut.FREE) == (s > 0)
    assert cut.BY_PLANE in seen
