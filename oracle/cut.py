"""FP64 CPU reference for cutting graph edges against obstacles: the Cut-QP
(eq. Cut-QP, Sec. III-B) and the cut heuristic of Alg. 2.  Test
infrastructure only: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py, never by the library.

One pair is an edge, given by the control points P ((p+1) x 3) of its Bezier
curve, and an obstacle O = {x : A x <= b}.  By the convex-hull property
(Property 1) the curve is free of O when conv(P) and O are disjoint; the
Cut-QP decides this: it minimises |delta|^2 over convex weights lambda and
slacks delta with A P lambda <= b + delta, and delta* = 0 exactly when the two
sets meet.

Obstacles here are axis-aligned boxes lo <= x <= hi (the paper's scenes are
built from boxes).  Then A = [I; -I], b = [hi; -lo], and for fixed
x = P lambda the best slack is delta = (A x - b)_+, whose squared norm is the
squared Euclidean distance from x to the box.  So |delta*|^2 is the squared
distance between conv(P) and the box, computed here as the distance from the
origin to the convex hull of the Minkowski difference {P_i - v_j} (v_j the
box corners): Qhull gives the hull, and the closest point is found by
projecting the origin onto every facet, edge and vertex and keeping the
nearest projection that lies in its simplex.

Alg. 2, in the paper's order, for one pair:
  1. some control point lies in O            -> 0 (the curve may collide);
  2. v_o = closestPoint(.), (h, l) = adjacentHyperplane(v_o); every control
     point strictly on the far side of the plane -> 1 (free);
  3. otherwise solve the Cut-QP: 1 if |delta*| > 0, else 0.
Reading of the unspecified helpers: closestPoint projects the centroid of
the control points onto O (for a box, a clamp); adjacentHyperplane is the
supporting plane of O with normal n = centroid - v_o, i.e. n.x = max over O of
n.x (for a box, the best corner), so O lies on its near side.  Step 2 uses
the strict inequality so that a curve touching O is left to step 3.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Tuple

import numpy as np
from scipy.optimize import linprog
from scipy.spatial import ConvexHull, QhullError

FREE, CUT = 1, 0
BY_POINT, BY_PLANE, BY_QP = 1, 2, 3
TAU = 1e-4   # margin of a certified classification (row-normalised LP slack)


def box_rows(lo, hi) -> Tuple[np.ndarray, np.ndarray]:
    """H-representation A x <= b of the box lo <= x <= hi."""
    A = np.concatenate([np.eye(3), -np.eye(3)])
    b = np.concatenate([np.asarray(hi, float), -np.asarray(lo, float)])
    return A, b


def box_corners(lo, hi) -> np.ndarray:
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return np.array([[(hi if (k >> c) & 1 else lo)[c] for c in range(3)] for k in range(8)])


def _closest_on_simplex(S: np.ndarray):
    """Closest point to the origin of the affine hull of the rows of S, with
    its affine weights; None when the rows are affinely dependent."""
    k = S.shape[0]
    if k == 1:
        return S[0].copy(), np.ones(1)
    D = S[1:] - S[0]
    M = D @ D.T
    if abs(np.linalg.det(M)) <= 1e-24 * max(1.0, np.abs(M).max()) ** (k - 1):
        return None
    t = np.linalg.solve(M, -D @ S[0])
    w = np.concatenate([[1.0 - t.sum()], t])
    return S[0] + t @ D, w


def min_distance_to_hull(W: np.ndarray) -> Tuple[float, np.ndarray]:
    """Squared distance from the origin to conv(W) (W: m x 3) and the closest
    point.  Exact up to rounding: Qhull's facets decide whether the origin is
    inside; otherwise every hull facet (triangle), hull edge and vertex is a
    candidate face, and the closest point is the nearest affine projection
    that lies inside its face."""
    W = np.asarray(W, float)
    try:
        hull = ConvexHull(W)
    except QhullError:
        hull = None
    if hull is not None:
        eq = hull.equations   # n.x + d <= 0 inside
        if np.all(eq[:, 3] <= 1e-12 * (1.0 + np.abs(W).max())):
            return 0.0, np.zeros(3)
        faces = set()
        for simp in hull.simplices:
            s = tuple(sorted(int(i) for i in simp))
            faces.add(s)
            for a in range(3):
                for c in range(a + 1, 3):
                    faces.add((s[a], s[c]))
        for i in hull.vertices:
            faces.add((int(i),))
    else:
        # flat (coplanar) point set: every triangle, segment and point
        m = W.shape[0]
        faces = {(i,) for i in range(m)}
        faces |= {(i, j) for i in range(m) for j in range(i + 1, m)}
        faces |= {(i, j, k) for i in range(m) for j in range(i + 1, m) for k in range(j + 1, m)}
    best, bx = np.inf, None
    for f in faces:
        r = _closest_on_simplex(W[list(f)])
        if r is None:
            continue
        x, w = r
        if np.all(w >= -1e-12):
            d = float(x @ x)
            if d < best:
                best, bx = d, x
    return best, bx


@dataclass
class CutQP:
    dist2: float            # |delta*|^2 = squared distance conv(P) <-> box
    x: np.ndarray           # closest point of conv(P)
    y: np.ndarray           # closest point of the box
    lam: np.ndarray         # convex weights with x = P^T lam
    delta: np.ndarray       # (A x - b)_+ (the Cut-QP slack at x)


def cut_qp(P, lo, hi) -> CutQP:
    """Optimum of the Cut-QP for a box obstacle (see the module text).  The
    closest point v of the Minkowski difference is x - y with x in conv(P)
    and y in the box; the convex weights of x come from the LP
    P^T lam - v in the box."""
    P = np.asarray(P, float)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    V = box_corners(lo, hi)
    Wd = (P[:, None, :] - V[None, :, :]).reshape(-1, 3)
    d2, v = min_distance_to_hull(Wd)
    lam = _weights_for(P, lo, hi, v)
    x = P.T @ lam
    A, b = box_rows(lo, hi)
    return CutQP(d2, x, x - v, lam, np.maximum(A @ x - b, 0.0))


def _weights_for(P, lo, hi, v) -> np.ndarray:
    """Convex weights lam with P^T lam - v in the box (exists at the optimum)."""
    m = P.shape[0]
    res = linprog(np.zeros(m), A_ub=np.concatenate([P.T, -P.T]),
                  b_ub=np.concatenate([hi + v, -(lo + v)]) + 1e-9,
                  A_eq=np.ones((1, m)), b_eq=[1.0], bounds=[(0, None)] * m, method="highs")
    if res.status != 0:
        return np.full(m, 1.0 / m)
    return res.x


def lp_margin(P, lo, hi) -> float:
    """s* = min over lam in the simplex of max_k (a_k.P lam - b_k) / |a_k|:
    s* < 0 when conv(P) reaches into the box's interior, > 0 when they are
    apart (an LP, the classification certificate used by the tests)."""
    P = np.asarray(P, float)
    A, b = box_rows(lo, hi)
    m = P.shape[0]
    # variables (lam, s): minimise s, A P^T lam - s <= b, sum lam = 1
    AP = A @ P.T
    c = np.zeros(m + 1); c[-1] = 1.0
    A_ub = np.concatenate([AP, -np.ones((6, 1))], axis=1)
    res = linprog(c, A_ub=A_ub, b_ub=b, A_eq=np.concatenate([np.ones((1, m)), np.zeros((1, 1))], axis=1),
                  b_eq=[1.0], bounds=[(0, None)] * m + [(None, None)], method="highs")
    return float(res.x[-1])


def closest_point(P, lo, hi) -> np.ndarray:
    """closestPoint of Alg. 2 (reading): the centroid of the control points
    projected onto the box."""
    return np.clip(np.asarray(P, float).mean(axis=0), lo, hi)


def adjacent_hyperplane(P, lo, hi, vo) -> Tuple[np.ndarray, float]:
    """adjacentHyperplane of Alg. 2 (reading): normal n = centroid - v_o and
    offset l = max over the box of n.x (the box lies in n.x <= l)."""
    n = np.asarray(P, float).mean(axis=0) - vo
    l = float(np.sum(np.where(n > 0, n * np.asarray(hi, float), n * np.asarray(lo, float))))
    return n, l


def heuristic(P, lo, hi, tol2: float = 0.0) -> Tuple[int, int, float]:
    """Alg. 2 for one (edge, box) pair: (code, step that decided, |delta*|^2
    when step 3 ran else NaN).  code 1 = free, 0 = may collide.  ``tol2`` is
    the squared slack counted as zero in step 3."""
    P = np.asarray(P, float)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    if np.any(np.all((P >= lo) & (P <= hi), axis=1)):
        return CUT, BY_POINT, np.nan
    vo = closest_point(P, lo, hi)
    n, l = adjacent_hyperplane(P, lo, hi, vo)
    if np.any(n != 0.0) and np.all(P @ n > l):
        return FREE, BY_PLANE, np.nan
    d2 = cut_qp(P, lo, hi).dist2
    return (FREE if d2 > tol2 else CUT), BY_QP, d2


# ---------------------------------------------------------------------------
# General convex polytope obstacles O = {x : A x <= b} (Assumption 1 of
# Sec. III-A: every obstacle is a convex polytope, given by n_c halfspaces).
#
# The Cut-QP is then  min |delta|^2  over convex weights lam and slacks delta
# with A P^T lam <= b + delta.  For fixed lam the best slack is
# delta = (M lam - b)_+ with M = A P^T (n_c x (p+1)), so the optimum is
#   v* = min over the simplex of f(lam) = |(M lam - b)_+|^2,
# a convex, continuously differentiable function; v* = 0 exactly when
# conv(P) and O meet.  Its Lagrange dual (multipliers mu >= 0 of the rows) is
#   max over mu >= 0 of  h(mu) = min_j mu . (M e_j - b) - |mu|^2 / 4,
# and h(mu) <= v* <= f(lam) for every mu >= 0 and every lam in the simplex
# (weak duality; equality at the optimum, where mu = 2 delta*).  The oracle
# returns v* enclosed by these two bounds.
# ---------------------------------------------------------------------------
@dataclass
class CutQPPoly:
    value: float            # f at the returned weights (upper bound of v*)
    lower: float            # dual bound h(mu) (lower bound of v*)
    lam: np.ndarray         # convex weights
    delta: np.ndarray       # (M lam - b)_+


def _project_simplex(v: np.ndarray) -> np.ndarray:
    """Euclidean projection onto {lam >= 0, sum lam = 1} (sort and threshold)."""
    u = np.sort(v)[::-1]
    css = np.cumsum(u) - 1.0
    k = np.arange(1, v.size + 1)
    rho = np.nonzero(u - css / k > 0)[0][-1]
    theta = css[rho] / (rho + 1.0)
    return np.maximum(v - theta, 0.0)


def poly_f(M, b, lam) -> float:
    r = np.maximum(M @ lam - b, 0.0)
    return float(r @ r)


def poly_dual(M, b, mu) -> float:
    """h(mu) = min_j mu . (M e_j - b) - |mu|^2 / 4 (a lower bound of the
    Cut-QP optimum for every mu >= 0)."""
    return float(np.min(mu @ (M - b[:, None])) - 0.25 * mu @ mu)


def poly_lp_margin(P, A, b) -> float:
    """s* = min over the simplex of max_k (a_k . P^T lam - b_k) / |a_k|: < 0
    when conv(P) reaches into the interior of O, > 0 when they are apart."""
    P, A, b = (np.asarray(a, float) for a in (P, A, b))
    nrm = np.linalg.norm(A, axis=1)
    AP = (A / nrm[:, None]) @ P.T
    m = P.shape[0]
    c = np.zeros(m + 1); c[-1] = 1.0
    res = linprog(c, A_ub=np.concatenate([AP, -np.ones((A.shape[0], 1))], axis=1), b_ub=b / nrm,
                  A_eq=np.concatenate([np.ones((1, m)), np.zeros((1, 1))], axis=1), b_eq=[1.0],
                  bounds=[(0, None)] * m + [(None, None)], method="highs")
    return float(res.x[-1])


def _refine(M, b, lam):
    """Exact minimiser on the pieces of the current point: with S the rows
    that are violated and J the weights that are positive, minimise
    |M_SJ lam_J - b_S|^2 subject to sum lam_J = 1 (a linear KKT system); the
    candidate is kept only when it stays in the simplex."""
    S = np.nonzero(M @ lam - b > 0)[0]
    J = np.nonzero(lam > 1e-13)[0]
    if S.size == 0 or J.size == 0:
        return lam
    MS = M[np.ix_(S, J)]
    k = J.size
    K = np.zeros((k + 1, k + 1))
    K[:k, :k] = 2.0 * MS.T @ MS
    K[:k, k] = 1.0
    K[k, :k] = 1.0
    rhs = np.concatenate([2.0 * MS.T @ b[S], [1.0]])
    try:
        sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    except np.linalg.LinAlgError:
        return lam
    cand = np.zeros_like(lam)
    cand[J] = sol[:k]
    if np.all(cand >= -1e-15):
        cand = np.maximum(cand, 0.0)
        cand /= cand.sum()
        return cand
    return lam


def cut_qp_poly(P, A, b) -> CutQPPoly:
    """Optimum of the Cut-QP for the obstacle {A x <= b}: zero (with the LP's
    common point) when conv(P) meets it; otherwise f minimised over the
    simplex by SLSQP from several starts, each result refined on its pieces
    (``_refine``); the best upper bound and the dual bound at mu = 2 delta
    enclose the optimum."""
    from scipy.optimize import minimize
    P, A, b = (np.asarray(a, float) for a in (P, A, b))
    M = A @ P.T
    m = P.shape[0]
    # common point: feasibility LP over the simplex
    res = linprog(np.zeros(m), A_ub=M, b_ub=b, A_eq=np.ones((1, m)), b_eq=[1.0],
                  bounds=[(0, None)] * m, method="highs")
    if res.status == 0:
        lam = _project_simplex(res.x)
        if poly_f(M, b, lam) == 0.0:
            return CutQPPoly(0.0, 0.0, lam, np.zeros(A.shape[0]))
    fun = lambda l: poly_f(M, b, l)
    jac = lambda l: 2.0 * M.T @ np.maximum(M @ l - b, 0.0)
    cons = [{"type": "eq", "fun": lambda l: np.sum(l) - 1.0, "jac": lambda l: np.ones(m)}]
    starts = [np.full(m, 1.0 / m)] + [np.eye(m)[j] for j in range(m)]
    best = None
    for x0 in starts:
        r = minimize(fun, x0, jac=jac, bounds=[(0, 1)] * m, constraints=cons, method="SLSQP",
                     options={"ftol": 1e-16, "maxiter": 500})
        lam = _project_simplex(r.x)
        for _ in range(3):
            lam = _refine(M, b, lam)
        if best is None or poly_f(M, b, lam) < poly_f(M, b, best):
            best = lam
    delta = np.maximum(M @ best - b, 0.0)
    return CutQPPoly(float(delta @ delta), poly_dual(M, b, 2.0 * delta), best, delta)


def poly_closest_point(P, A, b) -> np.ndarray:
    """closestPoint of Alg. 2 (reading) for a polytope: the point of O nearest
    the centroid of the control points (a strictly convex QP, solved by the
    primal active-set method from the LP's Chebyshev centre)."""
    from .qp import active_set
    P, A, b = (np.asarray(a, float) for a in (P, A, b))
    c = P.mean(axis=0)
    nrm = np.linalg.norm(A, axis=1)
    # Chebyshev centre: max r with A x + |a| r <= b
    res = linprog(np.array([0.0, 0.0, 0.0, -1.0]), A_ub=np.concatenate([A, nrm[:, None]], axis=1), b_ub=b,
                  bounds=[(None, None)] * 3 + [(0, None)], method="highs")
    x0 = res.x[:3]
    # min |x - c|^2 = x'x - 2 c'x + const: shift y = x - c so the objective is y'y
    r = active_set(np.eye(3), A, b - A @ c, np.zeros((0, 3)), np.zeros(0), x0 - c, [])
    return r.y + c


def poly_support(A, b, n) -> float:
    """max over O of n . x (an LP)."""
    res = linprog(-np.asarray(n, float), A_ub=A, b_ub=b, bounds=[(None, None)] * 3, method="highs")
    return float(-res.fun)


def heuristic_poly(P, A, b, tol2: float = 0.0):
    """Alg. 2 for one (edge, polytope) pair, as ``heuristic`` does for a box:
    (code, step that decided, Cut-QP value when step 3 ran else NaN)."""
    P, A, b = (np.asarray(a, float) for a in (P, A, b))
    if np.any(np.all(P @ A.T <= b, axis=1)):
        return CUT, BY_POINT, np.nan
    vo = poly_closest_point(P, A, b)
    n = P.mean(axis=0) - vo
    l = poly_support(A, b, n)
    if np.any(n != 0.0) and np.all(P @ n > l):
        return FREE, BY_PLANE, np.nan
    v = cut_qp_poly(P, A, b).value
    return (FREE if v > tol2 else CUT), BY_QP, v
