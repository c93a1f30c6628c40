"""Pins of the graph-building and adjacent-hyperplane oracle (Sec. III-A,
Thm. 2, Alg. 2) against facts that do not come from it: the cube-shaped
reachable set gives the Chebyshev-distance graph, a dense set of directions
sandwiches the Euclidean ball, symmetric rows give a symmetric graph, the
bit packing unpacks with numpy's own bit routine, and the nearest box and
its plane match brute force with an independent distance formula."""
import numpy as np

from oracle import graph as og
from workloads import gen


def test_cube_reach_is_chebyshev_graph():
    rng = np.random.default_rng(1)
    V = rng.uniform(0, 5, (300, 3))
    A = np.concatenate([np.eye(3), -np.eye(3)])
    g = 0.7
    adj = og.adjacency(V, -A, A, np.full(6, g))
    D = np.abs(V[:, None, :] - V[None, :, :]).max(axis=2)
    want = D <= g
    np.fill_diagonal(want, False)
    assert np.array_equal(adj, want)


def test_dense_directions_sandwich_the_ball():
    rng = np.random.default_rng(2)
    V = rng.uniform(0, 4, (300, 3))
    A = rng.standard_normal((400, 3))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    adj = og.adjacency(V, -A, A, np.ones(400))
    D = np.linalg.norm(V[:, None, :] - V[None, :, :], axis=2)
    off = ~np.eye(len(V), dtype=bool)
    assert np.all(adj[(D <= 1.0) & off])          # inside the ball: every row holds
    assert not np.any(adj[D > 1.5])               # 400 directions cover the sphere within 48 degrees


def test_symmetric_rows_give_a_symmetric_graph():
    rng = np.random.default_rng(3)
    V = rng.uniform(0, 4, (250, 3))
    A = rng.standard_normal((20, 3))
    A = np.concatenate([A, -A])
    g = np.tile(rng.uniform(0.8, 1.2, 20), 2)
    adj = og.adjacency(V, -A, A, g)
    assert np.array_equal(adj, adj.T) and not adj.diagonal().any() and adj.sum() > 0


def test_bit_packing_unpacks_with_numpy():
    rng = np.random.default_rng(4)
    adj = rng.random((77, 77)) < 0.2
    words = og.pack_bits(adj)
    bits = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")[:, :77]
    assert np.array_equal(bits.astype(bool), adj)


def test_adjacent_hyperplanes_brute_force():
    b = gen.gen_graph(n_nodes=400, n_obst=60)
    idx, pt, n, l = og.adjacent_hyperplanes(b.V, b.box_lo, b.box_hi)
    lo, hi = b.box_lo, b.box_hi
    for i in range(0, 400, 7):
        x = b.V[i]
        gap = np.maximum(np.maximum(lo - x, 0.0), x - hi)        # per-axis distance to each box
        d = np.sqrt((gap ** 2).sum(axis=1))
        assert abs(np.linalg.norm(x - pt[i]) - d.min()) <= 1e-12
        assert d[idx[i]] == d.min() and idx[i] == np.flatnonzero(d == d.min())[0]
        if d.min() > 0:
            corners = np.array([[(hi if (k >> c) & 1 else lo)[idx[i], c] for c in range(3)] for k in range(8)])
            assert np.all(corners @ n[i] <= l[i] + 1e-12) and n[i] @ x > l[i]
            assert abs(np.linalg.norm(n[i]) - 1) <= 1e-12


def test_workload_degree_and_order():
    b = gen.gen_graph(n_nodes=2000)
    adj = og.adjacency(b.V, b.F1, b.F2, b.G)
    deg = adj.sum(axis=1).mean()
    # 2,000 nodes in the 10 m cube: a reach of ~0.8 m gives about 1 edge per node
    assert 0.3 < deg < 5
    # Z-order numbering keeps consecutive nodes close
    step = np.linalg.norm(np.diff(b.V, axis=0), axis=1)
    assert np.median(step) < 2.0
