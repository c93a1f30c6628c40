"""GPU graph building (F1 v_i + F2 v_j <= G over all pairs) and adjacent
hyperplanes against the FP64 oracle, through the C ABI.

The adjacency is compared bit for bit on every pair whose value
max_k (F1 v_i + F2 v_j - G)_k is not within rounding of zero (both sides
compute it in FP64, in different orders); degrees are the popcounts of the
GPU's own rows.  The node numbering only decides which tiles are skipped,
so a permuted numbering must give the permuted graph."""
import numpy as np
import pytest
import torch

from oracle import graph as og
from workloads import gen

pytestmark = pytest.mark.gpu


def run_graph(b, V=None):
    from paper_2411_13507_amd.api import GraphGPU
    V = b.V if V is None else V
    g = GraphGPU(b, V.shape[0])
    adj, deg = g.run(torch.as_tensor(V, device=g.device))
    torch.cuda.synchronize()
    words = adj.cpu().numpy().view(np.uint32)
    out = np.unpackbits(words.view(np.uint8), axis=1, bitorder="little")[:, :V.shape[0]].astype(bool)
    g.close()
    return out, deg.cpu().numpy(), words


def compare(b, V, got, label):
    M = og.pair_values(V, b.F1, b.F2, b.G)
    want = og.adjacency(V, b.F1, b.F2, b.G)
    scale = 1.0 + np.abs(V).max() * (np.abs(b.F1).max() + np.abs(b.F2).max()) + np.abs(b.G).max()
    sure = np.abs(M) > 1e-12 * scale
    np.fill_diagonal(sure, True)
    bad = np.argwhere((got != want) & sure)
    print(f"{label}: {want.sum()} edges, {int((~sure).sum())} pairs within rounding of the boundary, "
          f"{len(bad)} mismatches", flush=True)
    assert len(bad) == 0, bad[:5]
    assert not got.diagonal().any()


def test_ragged_sizes_every_pair(gpu_available):
    for n in (1, 33, 64, 65, 700):
        b = gen.gen_graph(n_nodes=n, m=40)
        print(f"case: {n} nodes, 40 rows", flush=True)
        got, deg, words = run_graph(b)
        compare(b, b.V, got, f"n{n}")
        assert np.array_equal(deg, got.sum(axis=1))
        # bits past the last node stay clear
        if n % 32:
            assert np.all(words[:, -1] >> np.uint32(n % 32) == 0)


def test_full_size_graph(gpu_available):
    b = gen.gen_graph()
    print(f"case: {b.V.shape[0]} nodes, {b.F1.shape[0]} rows", flush=True)
    got, deg, _ = run_graph(b)
    compare(b, b.V, got, "graph5000")
    assert np.array_equal(deg, got.sum(axis=1))
    assert 30_000 < got.sum() < 70_000


def test_numbering_does_not_change_the_graph(gpu_available):
    """A random numbering defeats the tile skipping; the edges are the same."""
    b = gen.gen_graph(n_nodes=1500, m=64)
    got, _, _ = run_graph(b)
    perm = np.random.default_rng(8).permutation(len(b.V))
    got_p, _, _ = run_graph(b, V=b.V[perm])
    assert np.array_equal(got_p, got[np.ix_(perm, perm)])


def test_identical_nodes_and_generic_rows(gpu_available):
    """All nodes at one point with G > 0: every ordered pair but the self pairs
    is an edge; rows with independent F1, F2 and more than 64 rows (several
    LDS stages with a ragged last one)."""
    rng = np.random.default_rng(9)
    b = gen.GraphBatch(name="same", V=np.tile([[3.0, 4.0, 5.0]], (70, 1)), F1=rng.standard_normal((90, 3)),
                       F2=rng.standard_normal((90, 3)), G=np.full(90, 1e3), box_lo=np.zeros((0, 3)),
                       box_hi=np.zeros((0, 3)))
    got, deg, _ = run_graph(b)
    assert np.array_equal(got, ~np.eye(70, dtype=bool)) and np.all(deg == 69)
    b2 = gen.GraphBatch(name="generic", V=rng.uniform(0, 3, (300, 3)), F1=rng.standard_normal((90, 3)),
                        F2=rng.standard_normal((90, 3)), G=rng.uniform(2, 4, 90), box_lo=np.zeros((0, 3)),
                        box_hi=np.zeros((0, 3)))
    got2, _, _ = run_graph(b2)
    compare(b2, b2.V, got2, "generic")


def test_adjacent_hyperplanes(gpu_available):
    from paper_2411_13507_amd.api import adjacent_hyperplanes
    b = gen.gen_graph(n_nodes=5000)
    d = torch.device("cuda", 0)
    idx, point, plane = adjacent_hyperplanes(torch.as_tensor(b.V, device=d), torch.as_tensor(b.box_lo, device=d),
                                             torch.as_tensor(b.box_hi, device=d))
    torch.cuda.synchronize()
    w_idx, w_pt, w_n, w_l = og.adjacent_hyperplanes(b.V, b.box_lo, b.box_hi)
    idx, point, plane = idx.cpu().numpy(), point.cpu().numpy(), plane.cpu().numpy()
    # the nearest box is unique up to rounding of the distances
    C = np.clip(b.V[:, None, :], b.box_lo[None], b.box_hi[None])
    d2 = np.sort(np.sum((b.V[:, None, :] - C) ** 2, axis=2), axis=1)
    clear = d2[:, 1] - d2[:, 0] > 1e-12 * (1 + d2[:, 0])
    assert np.array_equal(idx[clear], w_idx[clear])
    assert np.abs(point[clear] - w_pt[clear]).max() <= 1e-12
    assert np.abs(plane[clear, :3] - w_n[clear]).max() <= 1e-12
    assert np.abs(plane[clear, 3] - w_l[clear]).max() <= 1e-11
    assert clear.mean() > 0.99


def test_graph_capture_replays(gpu_available):
    from paper_2411_13507_amd.api import GraphGPU
    b = gen.gen_graph(n_nodes=900)
    g = GraphGPU(b, 900)
    V = torch.as_tensor(b.V, device=g.device)
    adj, deg = g.run(V)
    torch.cuda.synchronize()
    ref = (adj.clone(), deg.clone())
    side = torch.cuda.Stream(device=g.device)
    side.wait_stream(torch.cuda.current_stream(g.device))
    with torch.cuda.stream(side):
        g.run(V, adj, deg)
    torch.cuda.current_stream(g.device).wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.run(V, adj, deg)
    for rep in range(3):
        adj.fill_(-1); deg.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(adj, ref[0]) and torch.equal(deg, ref[1]), rep
        g.run(V)
        torch.cuda.synchronize()
    g.close()
