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
