"""Pins of the path oracle (segments joined with C0/C1/C2 continuity).

Independent checks: a one-segment path equals the single-segment oracle; the
optimal curves are continuous in position, velocity and acceleration at the
joins (sampled with numpy's power-basis derivatives); a loose path is the
straight constant-speed line; the sampled curves stay in their polytopes and
within the derivative bounds; KKT residuals vanish."""
import numpy as np
import pytest
from numpy.polynomial import polynomial as npoly

from oracle import bezier, chain, qp, segment
from tests.test_bezier import power_basis
from workloads import gen


@pytest.fixture(scope="module")
def solved():
    b = gen.gen_cfg3(indices=range(12))
    out = []
    for i in range(b.n):
        ch = b.chain(i)
        out.append((ch, chain.solve(ch)))
    return out


def test_some_solved(solved):
    assert sum(r.status == qp.SOLVED for _, r in solved) >= 8


def test_joins_are_c2(solved):
    for ch, r in solved:
        if r.status != qp.SOLVED:
            continue
        T = ch["T"]
        for s in range(r.P.shape[0] - 1):
            a = power_basis(r.P[s], T)
            b = power_basis(r.P[s + 1], T)
            for order in (0, 1, 2):
                end = np.array([npoly.polyval(T, npoly.polyder(c, order)) for c in a])
                start = np.array([npoly.polyval(0.0, npoly.polyder(c, order)) for c in b])
                assert np.allclose(end, start, atol=1e-6 * (1 + np.abs(end).max())), (s, order)
        assert np.allclose(r.P[0, 0], ch["x0"][:3], atol=1e-12)
        assert np.allclose(r.P[-1, -1], ch["goal"], atol=1e-12)


def test_curves_satisfy_segment_constraints(solved):
    for ch, r in solved:
        if r.status != qp.SOLVED:
            continue
        T = ch["T"]
        t = np.linspace(0, T, 401)
        for s, sg in enumerate(ch["segments"]):
            pts = bezier.curve_bernstein(r.P[s], t, T)
            assert np.all(pts @ sg["A_face"].T <= sg["b_face"] + 1e-9)
            polys = power_basis(r.P[s], T)
            vel = np.stack([npoly.polyval(t, npoly.polyder(c, 1)) for c in polys], 1)
            acc = np.stack([npoly.polyval(t, npoly.polyder(c, 2)) for c in polys], 1)
            assert np.abs(vel).max() <= ch["vmax"] + 1e-7
            assert np.abs(acc).max() <= ch["amax"] + 1e-7
        assert r.kkt["max"] <= 1e-11


def test_one_segment_path_is_the_segment_problem():
    b = gen.gen_cfg1(indices=range(12))
    for i in range(b.n):
        inst = b.instance(i)
        ch = dict(p=inst["p"], T=inst["T"], vmax=inst["vmax"], amax=inst["amax"], x0=inst["x0"],
                  goal=inst["goal"], segments=[dict(A_face=inst["A_face"], b_face=inst["b_face"],
                                                    H=inst["H"], h0=inst["h0"], G=inst["G"])])
        a = segment.solve(inst)
        c = chain.solve(ch)
        assert a.status == c.status
        if a.status == qp.SOLVED:
            assert np.allclose(a.P, c.P[0], atol=1e-9)
            assert abs(a.cost - c.cost) <= 1e-9 * (1 + a.cost)


def test_loose_path_is_a_straight_line():
    """With inactive constraints the optimum of the summed energy is the
    constant-speed line from start to goal over the whole path."""
    rng = np.random.default_rng(0)
    S, p = 4, 7
    x0 = np.concatenate([rng.uniform(4, 6, 3), np.zeros(3)])
    goal = x0[:3] + rng.uniform(-2, 2, 3)
    segs = []
    for _ in range(S):
        H = rng.standard_normal((4, 3 * (p + 1)))
        H /= np.linalg.norm(H, axis=1, keepdims=True)
        segs.append(dict(A_face=np.concatenate([np.eye(3), -np.eye(3)]), b_face=np.full(6, 50.0),
                         H=H, h0=np.full(4, 1e4), G=np.zeros((4, 6))))
    ch = dict(p=p, T=1.0, vmax=10.0, amax=10.0, x0=x0, goal=goal, segments=segs)
    r = chain.solve(ch)
    assert r.status == qp.SOLVED and abs(r.cost) <= 1e-9
    tot = S * p
    for s in range(S):
        for k in range(p + 1):
            frac = (s * p + k) / tot
            assert np.allclose(r.P[s, k], x0[:3] + frac * (goal - x0[:3]), atol=1e-9)


def _join_state(P, T):
    """Start state (b(0), b'(0)) of one segment, from numpy's power basis
    (independent of the p/T (P_1 - P_0) formula the oracle rows use)."""
    polys = power_basis(P, T)
    pos = np.array([npoly.polyval(0.0, c) for c in polys])
    vel = np.array([npoly.polyval(0.0, npoly.polyder(c, 1)) for c in polys])
    return np.concatenate([pos, vel])


def _reach_residuals(ch, P):
    """H_s vec(P^s) - (h0_s + G_s x0_s) for every segment, with x0_s the
    path's start state for s = 0 and the power-basis join state otherwise."""
    out = []
    for s, sg in enumerate(ch["segments"]):
        xs = ch["x0"] if s == 0 else _join_state(P[s], ch["T"])
        out.append(sg["H"] @ P[s].ravel() - (sg["h0"] + sg["G"] @ xs))
    return out


def _flip_join_velocity_sign(c, ch):
    """A planted mistake on the CPU: the rows of every segment s >= 1 with the
    sign of the join velocity's p/T G[:, 3:] terms flipped."""
    p, T = ch["p"], ch["T"]
    nseg = 3 * (p + 1)
    A = c.A.copy()
    row = 0
    for s, sg in enumerate(ch["segments"]):
        nf = sg["A_face"].shape[0]
        row += nf * (p + 1) + 2 * 3 * p + 2 * 3 * (p - 1)
        r = sg["H"].shape[0]
        if s >= 1:
            off = s * nseg
            Gv = sg["G"][:, 3:]
            A[row:row + r, off + 3:off + 6] += 2 * p / T * Gv
            A[row:row + r, off:off + 3] -= 2 * p / T * Gv
        row += r
    assert row == A.shape[0]
    return A


def _solve_rows(c, A, ch):
    ph = qp.phase1(A, c.u, c.E, c.e, chain.y_bound(ch))
    if not (ph.feasible and ph.certified):
        return None
    r = qp.active_set(c.Q, A, c.u, c.E, c.e, ph.y, qp.initial_working_set(A, c.u, c.E, ph.y))
    return r.y.reshape(c.S, c.p + 1, 3) if r.status == qp.SOLVED else None


@pytest.fixture(scope="module")
def tightened_paths():
    """Solved paths with one reachable row of the second segment tightened
    below its value at the optimum: the new optimum is unique and differs,
    so that join-state row is active there (Thm. 2's rows for s >= 1 then
    decide the solution)."""
    b = gen.gen_cfg3(indices=range(10))
    out = []
    for i in range(b.n):
        ch = b.chain(i)
        r = chain.solve(ch)
        if r.status != qp.SOLVED or len(ch["segments"]) < 2:
            continue
        res = _reach_residuals(ch, r.P)[1]
        k = int(np.argmax(res))
        seg = dict(ch["segments"][1])
        seg["h0"] = seg["h0"].copy()
        seg["h0"][k] += res[k] - 0.05           # 0.05 below the row's value at the optimum
        ch2 = dict(ch, segments=[ch["segments"][0], seg] + ch["segments"][2:])
        r2 = chain.solve(ch2)
        if r2.status == qp.SOLVED:
            out.append((ch2, r2, k))
        if len(out) >= 4:
            break
    assert len(out) >= 3
    return out


def test_join_state_rows_hold_and_bind(tightened_paths):
    """On the oracle's optima every segment's reachable rows hold with the
    join state taken from the power basis, and the tightened row of segment
    1 holds with equality."""
    for ch, r, k in tightened_paths:
        res = _reach_residuals(ch, r.P)
        for s, v in enumerate(res):
            assert np.all(v <= 1e-9), (s, v.max())
        assert abs(res[1][k]) <= 1e-9, res[1][k]


def test_join_state_pin_catches_a_sign_error(tightened_paths):
    """The same check rejects the optima of the rows with the join
    velocity's sign flipped: a plausible mistake in them does not pass."""
    caught = 0
    for ch, _, k in tightened_paths:
        c = chain.build(ch)
        P = _solve_rows(c, _flip_join_velocity_sign(c, ch), ch)
        if P is None:
            caught += 1        # the mutant even changes the class
            continue
        res = _reach_residuals(ch, P)
        bad = any(np.any(v > 1e-7) for v in res) or abs(res[1][k]) > 1e-7
        caught += int(bad)
    assert caught == len(tightened_paths)
