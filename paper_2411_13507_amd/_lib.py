"""ctypes declarations of the C ABI in include/rbp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbp.so")

RBP_OK = 0
RBP_E_INVALID, RBP_E_SHAPE, RBP_E_ALLOC, RBP_E_DEVICE, RBP_E_STATE, RBP_E_SCRATCH = -1, -2, -3, -4, -5, -6
GRAPH_NOALLOC_DOUBLES = 1 << 20
SOLVED, INFEASIBLE, MAXITER, POLISH_FAILED, NUMERICAL, INVALID_INPUT = 0, 1, 2, 3, 4, 5

EXPORTED = (
    "rbp_default_opts", "rbp_build_batch", "rbp_batch_get_sizes", "rbp_solve_batch",
    "rbp_backward", "rbp_destroy_batch", "rbp_status_string",
    "rbp_build_chains", "rbp_chains_get_sizes", "rbp_solve_chains", "rbp_destroy_chains",
    "rbp_build_cut", "rbp_cut_run", "rbp_cut_qp_count", "rbp_destroy_cut",
    "rbp_build_graph", "rbp_graph_run", "rbp_destroy_graph", "rbp_graph_run_noalloc",
    "rbp_adjacent_hyperplanes",
    "rbp_build_mpc", "rbp_mpc_solve", "rbp_destroy_mpc",
)

_p = ctypes.c_void_p


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("n_instances", ctypes.c_int32), ("n_poly", ctypes.c_int32),
        ("degree", _p), ("T", _p), ("poly_off", _p), ("A_face", _p), ("b_face", _p),
        ("poly_idx", _p), ("reach_off", _p), ("H_off", _p), ("H", _p), ("h0", _p), ("G", _p),
        ("vmax", ctypes.c_double), ("amax", ctypes.c_double),
        ("n_reach", ctypes.c_int32), ("reach_idx", _p), ("pin_start_velocity", ctypes.c_int32),
    ]


class ChainDesc(ctypes.Structure):
    _fields_ = [
        ("n_chains", ctypes.c_int32), ("n_poly", ctypes.c_int32), ("degree", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("T", ctypes.c_double), ("vmax", ctypes.c_double),
        ("amax", ctypes.c_double), ("seg_off", _p), ("poly_off", _p), ("A_face", _p), ("b_face", _p),
        ("poly_idx", _p), ("reach_off", _p), ("H_off", _p), ("H", _p), ("h0", _p), ("G", _p),
    ]


class CutDesc(ctypes.Structure):
    _fields_ = [
        ("n_edges", ctypes.c_int32), ("n_obstacles", ctypes.c_int32), ("degree", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("box_lo", _p), ("box_hi", _p),
        ("n_polytopes", ctypes.c_int32), ("reserved2", ctypes.c_int32), ("pob_off", _p), ("pob_A", _p),
        ("pob_b", _p),
    ]


class GraphDesc(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int32), ("dim", ctypes.c_int32), ("n_rows", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("F1", _p), ("F2", _p), ("G", _p),
    ]


class MpcDesc(ctypes.Structure):
    _fields_ = [
        ("n_instances", ctypes.c_int32), ("horizon", ctypes.c_int32), ("n_reach", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("dt", ctypes.c_double), ("Q", ctypes.c_double * 36),
        ("R", ctypes.c_double * 9), ("w_length", ctypes.c_double), ("F1", _p), ("F2", _p), ("G", _p),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("admm_iters", ctypes.c_int32), ("rho", ctypes.c_float), ("alpha", ctypes.c_float),
        ("max_polish_steps", ctypes.c_int32), ("feas_tol", ctypes.c_double),
        ("kkt_tol", ctypes.c_double), ("store_for_backward", ctypes.c_int32), ("plain", ctypes.c_int32),
        ("launch_shape", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("debug_fill_lds", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class BatchSizes(ctypes.Structure):
    _fields_ = [
        ("n_instances", ctypes.c_int32), ("max_degree", ctypes.c_int32),
        ("points_total", ctypes.c_int64), ("faces_total", ctypes.c_int64),
    ]


class RbpError(RuntimeError):
    pass


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librbp.so (built in-tree by ``paper_2411_13507_amd.build``).  There
    is no fallback: a missing library is an error."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RbpError(f"{path} is missing: build it with `python -m paper_2411_13507_amd.build`")
    L = ctypes.CDLL(path)
    L.rbp_default_opts.argtypes = [ctypes.POINTER(SolveOpts)]
    L.rbp_default_opts.restype = None
    L.rbp_build_batch.argtypes = [ctypes.POINTER(ProblemDesc), _p, ctypes.POINTER(_p)]
    L.rbp_build_batch.restype = ctypes.c_int
    L.rbp_batch_get_sizes.argtypes = [_p, ctypes.POINTER(BatchSizes)]
    L.rbp_batch_get_sizes.restype = ctypes.c_int
    L.rbp_solve_batch.argtypes = [_p, _p, _p, _p, ctypes.POINTER(SolveOpts), _p, _p, _p, _p, _p, _p]
    L.rbp_solve_batch.restype = ctypes.c_int
    L.rbp_backward.argtypes = [_p, _p, _p, _p, _p, _p, _p, _p]
    L.rbp_backward.restype = ctypes.c_int
    L.rbp_destroy_batch.argtypes = [_p]
    L.rbp_destroy_batch.restype = None
    L.rbp_build_chains.argtypes = [ctypes.POINTER(ChainDesc), _p, ctypes.POINTER(_p)]
    L.rbp_build_chains.restype = ctypes.c_int
    L.rbp_chains_get_sizes.argtypes = [_p, ctypes.POINTER(BatchSizes)]
    L.rbp_chains_get_sizes.restype = ctypes.c_int
    L.rbp_solve_chains.argtypes = [_p, _p, _p, ctypes.POINTER(SolveOpts), _p, _p, _p, _p, _p, _p]
    L.rbp_solve_chains.restype = ctypes.c_int
    L.rbp_destroy_chains.argtypes = [_p]
    L.rbp_destroy_chains.restype = None
    L.rbp_build_cut.argtypes = [ctypes.POINTER(CutDesc), _p, ctypes.POINTER(_p)]
    L.rbp_build_cut.restype = ctypes.c_int
    L.rbp_cut_run.argtypes = [_p, _p, _p, _p, _p, _p, _p]
    L.rbp_cut_run.restype = ctypes.c_int
    L.rbp_cut_qp_count.argtypes = [_p, ctypes.POINTER(ctypes.c_int64)]
    L.rbp_cut_qp_count.restype = ctypes.c_int
    L.rbp_destroy_cut.argtypes = [_p]
    L.rbp_destroy_cut.restype = None
    L.rbp_build_graph.argtypes = [ctypes.POINTER(GraphDesc), _p, ctypes.POINTER(_p)]
    L.rbp_build_graph.restype = ctypes.c_int
    L.rbp_graph_run.argtypes = [_p, _p, _p, _p, _p]
    L.rbp_graph_run.restype = ctypes.c_int
    L.rbp_destroy_graph.argtypes = [_p]
    L.rbp_destroy_graph.restype = None
    L.rbp_graph_run_noalloc.argtypes = [ctypes.POINTER(GraphDesc), _p, _p, _p, _p]
    L.rbp_graph_run_noalloc.restype = ctypes.c_int
    L.rbp_adjacent_hyperplanes.argtypes = [ctypes.c_int32, _p, ctypes.c_int32, _p, _p, _p, _p, _p, _p]
    L.rbp_adjacent_hyperplanes.restype = ctypes.c_int
    L.rbp_build_mpc.argtypes = [ctypes.POINTER(MpcDesc), _p, ctypes.POINTER(_p)]
    L.rbp_build_mpc.restype = ctypes.c_int
    L.rbp_mpc_solve.argtypes = [_p, _p, _p, _p, ctypes.c_int32, ctypes.c_double, _p, _p, _p, _p, _p, _p, _p]
    L.rbp_mpc_solve.restype = ctypes.c_int
    L.rbp_destroy_mpc.argtypes = [_p]
    L.rbp_destroy_mpc.restype = None
    L.rbp_status_string.argtypes = [ctypes.c_int]
    L.rbp_status_string.restype = ctypes.c_char_p
    _LIB = L
    return L


def check(rc: int, what: str) -> None:
    if rc != RBP_OK:
        msg = load().rbp_status_string(rc).decode()
        raise RbpError(f"{what} failed: {rc} ({msg})")


def default_opts() -> SolveOpts:
    o = SolveOpts()
    load().rbp_default_opts(ctypes.byref(o))
    return o
