"""Bezier-curve mathematics for the FP64 CPU oracle (test infrastructure).

Sec. II-B of the paper: a curve of order ``p`` is ``b(t) = P z(t)`` with
``z`` the degree-``p`` Bernstein basis and ``P`` the ``p+1`` control points
(one column each); derivatives are linear maps of the control points, and the
curve stays in the convex hull of its control points (Property 1).  Here the
time interval is ``[0, T]`` and ``s = t / T``.

Nothing here is shared with the HIP path; this module is only imported by the
oracle, the tests and the benchmark's CPU baseline.
"""
from __future__ import annotations

from math import comb

import numpy as np


def bernstein(p: int, s) -> np.ndarray:
    """Bernstein basis values ``B_{i,p}(s) = C(p,i) s^i (1-s)^(p-i)``,
    shape ``(len(s), p+1)`` (closed form, Sec. II-B)."""
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    i = np.arange(p + 1)
    c = np.array([comb(p, k) for k in i], dtype=np.float64)
    return c[None, :] * s[:, None] ** i[None, :] * (1.0 - s[:, None]) ** (p - i)[None, :]


def curve_bernstein(P: np.ndarray, t, T: float = 1.0) -> np.ndarray:
    """Evaluate ``b(t)`` from control points ``P`` ((p+1) x d) by the closed form."""
    p = P.shape[0] - 1
    return bernstein(p, np.asarray(t, dtype=np.float64) / T) @ P


def decasteljau(P: np.ndarray, s: float) -> np.ndarray:
    """de Casteljau evaluation at parameter ``s`` in [0,1] (repeated linear
    interpolation of the control polygon)."""
    Q = np.array(P, dtype=np.float64, copy=True)
    n = Q.shape[0]
    for r in range(1, n):
        Q[: n - r] = (1.0 - s) * Q[: n - r] + s * Q[1 : n - r + 1]
    return Q[0]


def split(P: np.ndarray, s: float):
    """Subdivide a curve at ``s`` (Property 3): returns the control points of
    the two pieces, each re-parameterised over [0,1]."""
    Q = np.array(P, dtype=np.float64, copy=True)
    n = Q.shape[0]
    left, right = [Q[0].copy()], [Q[-1].copy()]
    for r in range(1, n):
        Q[: n - r] = (1.0 - s) * Q[: n - r] + s * Q[1 : n - r + 1]
        left.append(Q[0].copy())
        right.append(Q[n - r - 1].copy())
    return np.array(left), np.array(right[::-1])


def diff_matrix(p: int, order: int) -> np.ndarray:
    """Forward-difference operator of the given order on p+1 control points:
    ``(Delta^order P)_k``, shape ((p+1-order) x (p+1)).  Plain differences;
    the derivative scaling is applied by the caller."""
    D = np.eye(p + 1)
    for _ in range(order):
        D = D[1:] - D[:-1]
    return D


def derivative_points(P: np.ndarray, order: int, T: float = 1.0) -> np.ndarray:
    """Control points of the ``order``-th derivative curve (degree p-order):
    ``p!/(p-order)! / T^order * Delta^order P`` (the linear map of Sec. II-B)."""
    p = P.shape[0] - 1
    scale = 1.0
    for k in range(order):
        scale *= (p - k)
    return scale / T ** order * (diff_matrix(p, order) @ P)


def bernstein_gram(n: int) -> np.ndarray:
    """Gram matrix ``M[i,j] = int_0^1 B_{i,n} B_{j,n} ds
    = C(n,i) C(n,j) / ((2n+1) C(2n, i+j))`` (Beta-function integral)."""
    M = np.empty((n + 1, n + 1))
    for i in range(n + 1):
        for j in range(n + 1):
            M[i, j] = comb(n, i) * comb(n, j) / ((2 * n + 1) * comb(2 * n, i + j))
    return M


def hessian_1d(p: int, T: float = 1.0) -> np.ndarray:
    """``Q_1D`` with ``int_0^T |b''(t)|^2 dt = sum_c P[:,c]^T Q_1D P[:,c]``:
    ``b''`` has control points ``p(p-1)/T^2 Delta^2 P`` on the degree-(p-2)
    basis, and ``dt = T ds``."""
    D2 = diff_matrix(p, 2)
    return (p * (p - 1)) ** 2 / T ** 3 * (D2.T @ bernstein_gram(p - 2) @ D2)


def hessian(p: int, T: float = 1.0, d: int = 3) -> np.ndarray:
    """Full Hessian on point-major ``vec(P)``: ``Q_1D (x) I_d``."""
    return np.kron(hessian_1d(p, T), np.eye(d))


def path_length_bound(P: np.ndarray) -> float:
    """Property 2: sum of control-polygon edge lengths."""
    return float(np.linalg.norm(np.diff(P, axis=0), axis=1).sum())
