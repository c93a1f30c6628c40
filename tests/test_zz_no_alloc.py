"""The allocation-free graph run (rbp_graph_run_noalloc) against the graph
object's run (rbp_build_graph + rbp_graph_run) on the same nodes: identical
adjacency bits and degrees, on two calls in a row, the second with fewer
nodes (the fixed workspace keeps the first call's contents)."""
import pytest
import torch

from paper_2411_13507_amd import _lib
from paper_2411_13507_amd.api import GraphGPU, graph_run_noalloc
from workloads import gen

pytestmark = pytest.mark.gpu


def _reference(problem, V):
    g = GraphGPU(problem, V.shape[0], device="cuda:0")
    try:
        adj, deg = g.run(V)
        torch.cuda.synchronize()
        return adj.clone(), deg.clone()
    finally:
        g.close()


def test_noalloc_matches_graph_object_twice(gpu_available):
    dev = torch.device("cuda", 0)
    gb = gen.gen_graph()                      # 5,000 nodes, 64 rows
    F1, F2, G = (torch.as_tensor(a, device=dev) for a in (gb.F1, gb.F2, gb.G))
    cases = [torch.as_tensor(gb.V, device=dev),                      # 5,000 nodes
             torch.as_tensor(gb.V[1234:1234 + 777].copy(), device=dev)]  # then 777
    for k, V in enumerate(cases):
        print(f"noalloc case {k}: {V.shape[0]} nodes", flush=True)
        adj, deg = graph_run_noalloc(F1, F2, G, V)
        torch.cuda.synchronize()
        ref_adj, ref_deg = _reference(gb, V)
        assert torch.equal(adj, ref_adj), k
        assert torch.equal(deg, ref_deg), k
        assert int(deg.sum()) > 0


def test_noalloc_rejects_oversized_problem(gpu_available):
    dev = torch.device("cuda", 0)
    gb = gen.gen_graph(n_nodes=64, m=64)
    F1, F2, G = (torch.as_tensor(a, device=dev) for a in (gb.F1, gb.F2, gb.G))
    V = torch.zeros((9000, 3), dtype=torch.float64, device=dev)   # 2 n m > 2^20
    with pytest.raises(_lib.RbpError, match="-6"):
        graph_run_noalloc(F1, F2, G, V)
