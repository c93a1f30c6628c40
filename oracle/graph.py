"""FP64 CPU reference for building the graph of Bezier curves and for the
adjacent hyperplanes of its nodes (Sec. III-A, Thm. 2, Alg. 2, Sec. III-D).
Test infrastructure only: imported by tests/ and the CPU-baseline leg of
bench.py, never by the library.

buildGraph: with the reachable-polytope pair (F, G) of Theorem 2, nodes v_i
and v_j are joined by an edge when F [v_i; v_j] <= G (every row).  F is split
into the columns acting on the start (F1) and on the end (F2), so the test
for the ordered pair (i, j) reads  max_k (F1 v_i + F2 v_j - G)_k <= 0.  A node
is not joined to itself.

adjacentHyperplane (reading, as in the graph cut): for a node x, the point of
the nearest obstacle closest to x (for a box, the clamp of x; nearest box by
Euclidean distance, lowest index on ties) and the plane through it with unit
normal n = (x - v_o) / |x - v_o|: the obstacle lies in n.y <= n.v_o and x on
the far side.  A node inside an obstacle has no such plane (distance 0).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def pair_values(V, F1, F2, G) -> np.ndarray:
    """M[i, j] = max_k (F1 v_i + F2 v_j - G)_k for every ordered pair."""
    V = np.asarray(V, float)
    A = V @ np.asarray(F1, float).T            # [N, m]
    B = V @ np.asarray(F2, float).T - np.asarray(G, float)
    N = V.shape[0]
    M = np.empty((N, N))
    step = max(1, 4_000_000 // (N * A.shape[1] + 1))
    for s in range(0, N, step):
        M[s:s + step] = np.max(A[s:s + step, None, :] + B[None, :, :], axis=2)
    return M


def adjacency(V, F1, F2, G) -> np.ndarray:
    """Boolean [N, N]: edge i -> j when F [v_i; v_j] <= G, i != j."""
    M = pair_values(V, F1, F2, G)
    adj = M <= 0.0
    np.fill_diagonal(adj, False)
    return adj


def pack_bits(adj: np.ndarray) -> np.ndarray:
    """Row-major bitmask [N, ceil(N/32)] uint32: bit j % 32 of word j // 32."""
    N = adj.shape[0]
    W = (N + 31) // 32
    out = np.zeros((N, W), dtype=np.uint32)
    for w in range(W):
        blk = adj[:, 32 * w:32 * (w + 1)].astype(np.uint64)
        out[:, w] = (blk << np.arange(blk.shape[1], dtype=np.uint64)).sum(axis=1).astype(np.uint32)
    return out


def adjacent_hyperplanes(V, lo, hi) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Per node: index of the nearest box, the closest point on it, the unit
    normal n and offset l of the separating plane (obstacle in n.y <= l, node
    in n.x > l); n = 0, l = 0 for a node inside a box."""
    V = np.asarray(V, float)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    C = np.clip(V[:, None, :], lo[None], hi[None])      # [N, O, 3]
    d2 = np.sum((V[:, None, :] - C) ** 2, axis=2)
    idx = np.argmin(d2, axis=1)
    pt = C[np.arange(len(V)), idx]
    diff = V - pt
    nrm = np.linalg.norm(diff, axis=1)
    n = np.where(nrm[:, None] > 0, diff / np.where(nrm > 0, nrm, 1.0)[:, None], 0.0)
    l = np.sum(n * pt, axis=1)
    return idx, pt, n, l
