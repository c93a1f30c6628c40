"""Python face of the C ABI: device memory and streams come from PyTorch,
every step of the computation runs in librbp.so."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(a, dtype, device) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device).contiguous()


def _check_out(owner, specs, device) -> None:
    """Every (tensor, dtype, numel) of a caller-supplied output set must be a
    contiguous tensor of that type and size on ``device``: the library
    writes through the raw pointers."""
    for t, dtype, n in specs:
        if t.dtype != dtype or not t.is_contiguous() or t.numel() != n or t.device != device:
            raise ValueError(f"{type(owner).__name__}: output of {t.numel()} {t.dtype} on {t.device}, "
                             f"expected {n} contiguous {dtype} on {device}")


@dataclass
class SolveResult:
    P: torch.Tensor          # [3 * points_total] float64
    cost: torch.Tensor       # [N]
    status: torch.Tensor     # [N] int32
    kkt: torch.Tensor        # [N]
    iters: torch.Tensor      # [N, 2] int32


@dataclass
class Gradients:
    x0: torch.Tensor         # [N, 6]
    goal: torch.Tensor       # [N, 3]
    b_inst: torch.Tensor     # [faces_total] per-instance face gradients
    flags: torch.Tensor      # [N] int32


class SegmentBatchGPU:
    """A built batch of segment problems resident on one GPU.

    ``problem`` is any object with the array attributes of the C description
    (degree, T, poly_off, A_face, b_face, poly_idx, reach_off, H_off, H, h0,
    G, vmax, amax), for instance a ``workloads.gen.SegmentBatch``.  An
    optional ``reach_idx`` attribute (not None) selects the shared-table form
    of the reachable rows: reach_off / H_off then index a table of blocks and
    instance i uses block reach_idx[i].  ``pin_v0`` (if true) pins the start
    velocity as well: (p/T)(P_1 - P_0) = x0[3:6].
    """

    def __init__(self, problem, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise _lib.RbpError("no GPU visible: the batched segment-QP library runs only on the GPU")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        L = _lib.load()
        f64, i32, i64 = torch.float64, torch.int32, torch.int64
        d = self.device
        self.degree = _dev(problem.degree, i32, d)
        self.T = _dev(problem.T, f64, d)
        self.poly_off = _dev(problem.poly_off, i32, d)
        self.A_face = _dev(problem.A_face, f64, d)
        self.b_face = _dev(problem.b_face, f64, d)
        self.poly_idx = _dev(problem.poly_idx, i32, d)
        self.reach_off = _dev(problem.reach_off, i64, d)
        self.H_off = _dev(problem.H_off, i64, d)
        self.H = _dev(problem.H, f64, d)
        self.h0 = _dev(problem.h0, f64, d)
        self.G = _dev(np.asarray(problem.G).reshape(-1), f64, d)
        self.N = int(self.degree.numel())
        ridx = getattr(problem, "reach_idx", None)
        self.reach_idx = None if ridx is None else _dev(ridx, i32, d)
        desc = _lib.ProblemDesc(
            self.N, int(self.poly_off.numel()) - 1,
            _ptr(self.degree), _ptr(self.T), _ptr(self.poly_off), _ptr(self.A_face), _ptr(self.b_face),
            _ptr(self.poly_idx), _ptr(self.reach_off), _ptr(self.H_off), _ptr(self.H), _ptr(self.h0),
            _ptr(self.G), float(problem.vmax), float(problem.amax),
            0 if ridx is None else int(self.reach_off.numel()) - 1, _ptr(self.reach_idx),
            1 if getattr(problem, "pin_v0", False) else 0,
        )
        h = ctypes.c_void_p()
        with torch.cuda.device(d):
            _lib.check(L.rbp_build_batch(ctypes.byref(desc), _stream_handle(d), ctypes.byref(h)), "rbp_build_batch")
        self._h = h
        # incremented by every forward pass: the library keeps the state of the
        # last one only (the autograd node checks it before differentiating)
        self.forward_generation = 0
        sz = _lib.BatchSizes()
        _lib.check(L.rbp_batch_get_sizes(h, ctypes.byref(sz)), "rbp_batch_get_sizes")
        self.points_total = int(sz.points_total)
        self.faces_total = int(sz.faces_total)
        self.max_degree = int(sz.max_degree)
        deg = np.asarray(problem.degree, np.int64)
        self.pt_off = np.concatenate([[0], np.cumsum(deg + 1)])
        nf = np.diff(np.asarray(problem.poly_off, np.int64))[np.asarray(problem.poly_idx, np.int64)]
        self.face_off = np.concatenate([[0], np.cumsum(nf)])
        # face-table index of every per-instance face gradient (for scatter-add)
        po = np.asarray(problem.poly_off, np.int64)[np.asarray(problem.poly_idx, np.int64)]
        self.face_index = torch.as_tensor(
            np.concatenate([np.arange(a, a + k) for a, k in zip(po, nf)]) if len(nf) else np.zeros(0, np.int64),
            dtype=torch.int64, device=d)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().rbp_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc_outputs(self) -> SolveResult:
        d, N = self.device, self.N
        return SolveResult(
            P=torch.empty(3 * self.points_total, dtype=torch.float64, device=d),
            cost=torch.empty(N, dtype=torch.float64, device=d),
            status=torch.empty(N, dtype=torch.int32, device=d),
            kkt=torch.empty(N, dtype=torch.float64, device=d),
            iters=torch.zeros((N, 2), dtype=torch.int32, device=d),
        )

    def solve(self, x0: torch.Tensor, goal: torch.Tensor, b_face: Optional[torch.Tensor] = None,
              opts: Optional[_lib.SolveOpts] = None, out: Optional[SolveResult] = None) -> SolveResult:
        """Forward pass (rbp_solve_batch) on the current torch stream."""
        o = out or self.alloc_outputs()
        opts = opts or _lib.default_opts()
        for t, shape in ((x0, (self.N, 6)), (goal, (self.N, 3))):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape or t.device != self.device:
                raise ValueError(f"expected contiguous float64 {shape} on {self.device}")
        if b_face is not None and (b_face.dtype != torch.float64 or not b_face.is_contiguous()
                                   or b_face.numel() != self.b_face.numel() or b_face.device != self.device):
            raise ValueError(f"b_face must be a contiguous float64 tensor shaped like the face table on {self.device}")
        _check_out(o, ((o.P, torch.float64, 3 * self.points_total), (o.cost, torch.float64, self.N),
                       (o.status, torch.int32, self.N), (o.kkt, torch.float64, self.N),
                       (o.iters, torch.int32, 2 * self.N)), self.device)
        self.forward_generation += 1
        rc = _lib.load().rbp_solve_batch(
            self._h, _ptr(x0), _ptr(goal), _ptr(b_face), ctypes.byref(opts), _ptr(o.P), _ptr(o.cost),
            _ptr(o.status), _ptr(o.kkt), _ptr(o.iters), _stream_handle(self.device))
        _lib.check(rc, "rbp_solve_batch")
        return o

    def backward(self, grad_P: Optional[torch.Tensor] = None, grad_cost: Optional[torch.Tensor] = None,
                 out: Optional[Gradients] = None) -> Gradients:
        """Implicit-KKT vector-Jacobian product of the last forward pass."""
        d, N = self.device, self.N
        for t, n, name in ((grad_P, 3 * self.points_total, "grad_P"), (grad_cost, N, "grad_cost")):
            if t is not None and (t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != n
                                  or t.device != d):
                raise ValueError(f"{name} must be a contiguous float64 tensor of {n} elements on {d}")
        g = out or Gradients(
            x0=torch.empty((N, 6), dtype=torch.float64, device=d),
            goal=torch.empty((N, 3), dtype=torch.float64, device=d),
            b_inst=torch.empty(self.faces_total, dtype=torch.float64, device=d),
            flags=torch.empty(N, dtype=torch.int32, device=d),
        )
        _check_out(g, ((g.x0, torch.float64, 6 * N), (g.goal, torch.float64, 3 * N),
                       (g.b_inst, torch.float64, self.faces_total), (g.flags, torch.int32, N)), d)
        rc = _lib.load().rbp_backward(
            self._h, _ptr(grad_P), _ptr(grad_cost), _ptr(g.x0), _ptr(g.goal), _ptr(g.b_inst), _ptr(g.flags),
            _stream_handle(d))
        _lib.check(rc, "rbp_backward")
        return g

    def P_of(self, P_flat: torch.Tensor, i: int) -> torch.Tensor:
        a, b = self.pt_off[i], self.pt_off[i + 1]
        return P_flat[3 * a:3 * b].view(-1, 3)


class ChainBatchGPU:
    """A built batch of multi-segment paths (degree-7 segments joined with
    continuous position, velocity and acceleration) on one GPU.

    ``problem`` has the array attributes of the C path description
    (seg_off, poly_off, A_face, b_face, poly_idx, reach_off, H_off, H, h0, G)
    and scalars degree, T, vmax, amax, e.g. ``workloads.gen.ChainBatch``.
    """

    def __init__(self, problem, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise _lib.RbpError("no GPU visible: the path solver runs only on the GPU")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        L = _lib.load()
        f64, i32, i64 = torch.float64, torch.int32, torch.int64
        d = self.device
        self.seg_off = _dev(problem.seg_off, i64, d)
        self.poly_off = _dev(problem.poly_off, i32, d)
        self.A_face = _dev(problem.A_face, f64, d)
        self.b_face = _dev(problem.b_face, f64, d)
        self.poly_idx = _dev(problem.poly_idx, i32, d)
        self.reach_off = _dev(problem.reach_off, i64, d)
        self.H_off = _dev(problem.H_off, i64, d)
        self.H = _dev(problem.H, f64, d)
        self.h0 = _dev(problem.h0, f64, d)
        self.G = _dev(np.asarray(problem.G).reshape(-1), f64, d)
        self.N = int(self.seg_off.numel()) - 1
        self.degree = int(problem.degree)
        desc = _lib.ChainDesc(
            self.N, int(self.poly_off.numel()) - 1, self.degree, 0, float(problem.T), float(problem.vmax),
            float(problem.amax), _ptr(self.seg_off), _ptr(self.poly_off), _ptr(self.A_face), _ptr(self.b_face),
            _ptr(self.poly_idx), _ptr(self.reach_off), _ptr(self.H_off), _ptr(self.H), _ptr(self.h0), _ptr(self.G))
        h = ctypes.c_void_p()
        with torch.cuda.device(d):
            _lib.check(L.rbp_build_chains(ctypes.byref(desc), _stream_handle(d), ctypes.byref(h)), "rbp_build_chains")
        self._h = h
        sz = _lib.BatchSizes()
        _lib.check(L.rbp_chains_get_sizes(h, ctypes.byref(sz)), "rbp_chains_get_sizes")
        self.points_total = int(sz.points_total)
        self.seg_off_host = np.asarray(problem.seg_off, np.int64)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().rbp_destroy_chains(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, x0: torch.Tensor, goal: torch.Tensor, opts: Optional[_lib.SolveOpts] = None,
              out: Optional[SolveResult] = None) -> SolveResult:
        d, N = self.device, self.N
        o = out or SolveResult(
            P=torch.empty(3 * self.points_total, dtype=torch.float64, device=d),
            cost=torch.empty(N, dtype=torch.float64, device=d),
            status=torch.empty(N, dtype=torch.int32, device=d),
            kkt=torch.empty(N, dtype=torch.float64, device=d),
            iters=torch.zeros((N, 2), dtype=torch.int32, device=d))
        for t, shape in ((x0, (N, 6)), (goal, (N, 3))):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape or t.device != d:
                raise ValueError(f"expected contiguous float64 {shape} on {d}")
        opts = opts or _lib.default_opts()
        rc = _lib.load().rbp_solve_chains(self._h, _ptr(x0), _ptr(goal), ctypes.byref(opts), _ptr(o.P),
                                          _ptr(o.cost), _ptr(o.status), _ptr(o.kkt), _ptr(o.iters),
                                          _stream_handle(d))
        _lib.check(rc, "rbp_solve_chains")
        return o


@dataclass
class CutResult:
    code: torch.Tensor        # [n_obstacles, n_edges] uint8: 1 free, 0 may collide
    step: torch.Tensor        # [n_obstacles, n_edges] uint8: step of Alg. 2 that decided
    qp_dist2: torch.Tensor    # [n_obstacles, n_edges] float64: |delta*|^2 where step 3 ran, NaN elsewhere
    n_collide: torch.Tensor   # [n_edges] int32: obstacles the edge may collide with


class CutGPU:
    """Graph edges cut against convex obstacles on one GPU (Alg. 2 with the
    Cut-QP for the undecided pairs).  ``problem`` has box_lo and box_hi
    ([n_boxes, 3]), optionally polytopes (pob_off [n_poly+1], pob_A [rows, 3],
    pob_b [rows]; numbered after the boxes) and degree, e.g.
    ``workloads.gen.CutBatch``; the edges' control points are passed to each
    run."""

    def __init__(self, problem, n_edges: int, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise _lib.RbpError("no GPU visible: the cut kernels run only on the GPU")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        L = _lib.load()
        d = self.device
        self.box_lo = _dev(problem.box_lo, torch.float64, d)
        self.box_hi = _dev(problem.box_hi, torch.float64, d)
        pob_off = getattr(problem, "pob_off", None)
        n_poly = 0 if pob_off is None else int(len(pob_off) - 1)
        if n_poly > 0:
            self.pob_off = _dev(np.asarray(pob_off), torch.int32, d)
            self.pob_A = _dev(problem.pob_A, torch.float64, d)
            self.pob_b = _dev(problem.pob_b, torch.float64, d)
        n_box = int(self.box_lo.shape[0])
        self.n_edges, self.n_obst, self.degree = int(n_edges), n_box + n_poly, int(problem.degree)
        desc = _lib.CutDesc(self.n_edges, n_box, self.degree, 0, _ptr(self.box_lo), _ptr(self.box_hi), n_poly, 0,
                            _ptr(self.pob_off) if n_poly else None, _ptr(self.pob_A) if n_poly else None,
                            _ptr(self.pob_b) if n_poly else None)
        h = ctypes.c_void_p()
        with torch.cuda.device(d):
            _lib.check(L.rbp_build_cut(ctypes.byref(desc), _stream_handle(d), ctypes.byref(h)), "rbp_build_cut")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().rbp_destroy_cut(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self) -> CutResult:
        d, E, O = self.device, self.n_edges, self.n_obst
        return CutResult(code=torch.empty((O, E), dtype=torch.uint8, device=d),
                         step=torch.empty((O, E), dtype=torch.uint8, device=d),
                         qp_dist2=torch.empty((O, E), dtype=torch.float64, device=d),
                         n_collide=torch.empty(E, dtype=torch.int32, device=d))

    def run(self, P: torch.Tensor, out: Optional[CutResult] = None, with_step: bool = True,
            with_dist: bool = True) -> CutResult:
        """Classify every (edge, obstacle) pair; P is [n_edges, degree+1, 3]
        float64 on the device."""
        o = out or self.alloc()
        P = P.contiguous()
        rc = _lib.load().rbp_cut_run(self._h, _ptr(P), _ptr(o.code), _ptr(o.step) if with_step else None,
                                     _ptr(o.qp_dist2) if with_dist else None, _ptr(o.n_collide),
                                     _stream_handle(self.device))
        _lib.check(rc, "rbp_cut_run")
        return o

    def qp_count(self) -> int:
        """Pairs the last run sent to the Cut-QP (synchronises)."""
        v = ctypes.c_int64()
        _lib.check(_lib.load().rbp_cut_qp_count(self._h, ctypes.byref(v)), "rbp_cut_qp_count")
        return int(v.value)


class GraphGPU:
    """Edges of the graph of Bezier curves on one GPU (F1 v_i + F2 v_j <= G).
    ``problem`` has F1 [m, d], F2 [m, d] and G [m], e.g.
    ``workloads.gen.GraphBatch``; nodes are passed to each run."""

    def __init__(self, problem, n_nodes: int, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise _lib.RbpError("no GPU visible: the graph kernels run only on the GPU")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        d = self.device
        self.F1 = _dev(problem.F1, torch.float64, d)
        self.F2 = _dev(problem.F2, torch.float64, d)
        self.G = _dev(problem.G, torch.float64, d)
        self.n_nodes, self.m, self.dim = int(n_nodes), int(self.F1.shape[0]), int(self.F1.shape[1])
        desc = _lib.GraphDesc(self.n_nodes, self.dim, self.m, 0, _ptr(self.F1), _ptr(self.F2), _ptr(self.G))
        h = ctypes.c_void_p()
        with torch.cuda.device(d):
            _lib.check(_lib.load().rbp_build_graph(ctypes.byref(desc), _stream_handle(d), ctypes.byref(h)),
                       "rbp_build_graph")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().rbp_destroy_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, V: torch.Tensor, adj: Optional[torch.Tensor] = None, degree: Optional[torch.Tensor] = None):
        """Adjacency bitmask [n, ceil(n/32)] (int32 tensor holding uint32 words)
        and out-degrees [n] of the nodes V [n, d] (float64, on the device)."""
        n, d = self.n_nodes, self.device
        adj = adj if adj is not None else torch.empty((n, (n + 31) // 32), dtype=torch.int32, device=d)
        degree = degree if degree is not None else torch.empty(n, dtype=torch.int32, device=d)
        V = V.contiguous()
        _lib.check(_lib.load().rbp_graph_run(self._h, _ptr(V), _ptr(adj), _ptr(degree), _stream_handle(d)),
                   "rbp_graph_run")
        return adj, degree


def graph_run_noalloc(F1: torch.Tensor, F2: torch.Tensor, G: torch.Tensor, V: torch.Tensor,
                      adj: Optional[torch.Tensor] = None, degree: Optional[torch.Tensor] = None):
    """Adjacency and out-degrees as ``GraphGPU.run``, through the entry point
    that allocates no device memory (its workspace is a fixed per-GPU array
    in the library).  F1, F2 [m, d], G [m], V [n, d]: float64 tensors on one
    GPU.  With ``adj`` and ``degree`` given (int32, [n, ceil(n/32)] and [n])
    nothing is allocated at all."""
    d = V.device
    if d.type != "cuda":
        raise _lib.RbpError("graph_run_noalloc needs device tensors")
    for name, t in (("F1", F1), ("F2", F2), ("G", G), ("V", V)):
        if t.device != d or t.dtype != torch.float64 or not t.is_contiguous():
            raise _lib.RbpError(f"{name} must be a contiguous float64 tensor on {d}")
    m, dim = int(F1.shape[0]), int(F1.shape[1])
    n = int(V.shape[0])
    if tuple(F2.shape) != (m, dim) or tuple(G.shape) != (m,) or tuple(V.shape) != (n, dim):
        raise _lib.RbpError("shapes of F1, F2, G, V disagree")
    adj = adj if adj is not None else torch.empty((n, (n + 31) // 32), dtype=torch.int32, device=d)
    degree = degree if degree is not None else torch.empty(n, dtype=torch.int32, device=d)
    if adj.device != d or adj.dtype != torch.int32 or tuple(adj.shape) != (n, (n + 31) // 32) \
            or not adj.is_contiguous():
        raise _lib.RbpError("adj must be a contiguous int32 [n, ceil(n/32)] tensor on the device of V")
    if degree.device != d or degree.dtype != torch.int32 or tuple(degree.shape) != (n,):
        raise _lib.RbpError("degree must be an int32 [n] tensor on the device of V")
    desc = _lib.GraphDesc(n, dim, m, 0, _ptr(F1), _ptr(F2), _ptr(G))
    with torch.cuda.device(d):
        _lib.check(_lib.load().rbp_graph_run_noalloc(ctypes.byref(desc), _ptr(V), _ptr(adj), _ptr(degree),
                                                     _stream_handle(d)), "rbp_graph_run_noalloc")
    return adj, degree


def adjacent_hyperplanes(X: torch.Tensor, box_lo: torch.Tensor, box_hi: torch.Tensor):
    """Nearest box, closest point and separating plane (n, l) per node;
    tensors on the device (float64)."""
    n, d = int(X.shape[0]), X.device
    idx = torch.empty(n, dtype=torch.int32, device=d)
    point = torch.empty((n, 3), dtype=torch.float64, device=d)
    plane = torch.empty((n, 4), dtype=torch.float64, device=d)
    X, box_lo, box_hi = X.contiguous(), box_lo.contiguous(), box_hi.contiguous()
    _lib.check(_lib.load().rbp_adjacent_hyperplanes(n, _ptr(X), int(box_lo.shape[0]), _ptr(box_lo), _ptr(box_hi),
                                                    _ptr(idx), _ptr(point), _ptr(plane), _stream_handle(d)),
               "rbp_adjacent_hyperplanes")
    return idx, point, plane


@dataclass
class MpcResult:
    X: torch.Tensor          # [n, N+1, 6] float64
    U: torch.Tensor          # [n, N, 3]
    cost: torch.Tensor       # [n]
    status: torch.Tensor     # [n] int32
    kkt: torch.Tensor        # [n]
    iters: torch.Tensor      # [n] int32


class MpcGPU:
    """Batched MPC refinement (eq. MPC) resident on one GPU.  ``problem``
    has the shared attributes of ``workloads.gen.MpcBatch`` (N, dt, Q, R, w,
    F1, F2, G); ``n`` is the number of instances per call."""

    def __init__(self, problem, n: int, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise _lib.RbpError("no GPU visible: the MPC solver runs only on the GPU")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        L = _lib.load()
        d = self.device
        self.n, self.N = int(n), int(problem.N)
        self.F1 = _dev(np.asarray(problem.F1).reshape(-1), torch.float64, d)
        self.F2 = _dev(np.asarray(problem.F2).reshape(-1), torch.float64, d)
        self.G = _dev(problem.G, torch.float64, d)
        desc = _lib.MpcDesc()
        desc.n_instances, desc.horizon, desc.n_reach, desc.reserved = self.n, self.N, int(self.G.numel()), 0
        desc.dt = float(problem.dt)
        desc.Q[:] = [float(v) for v in np.asarray(problem.Q, float).ravel()]
        desc.R[:] = [float(v) for v in np.asarray(problem.R, float).ravel()]
        desc.w_length = float(problem.w)
        desc.F1, desc.F2, desc.G = _ptr(self.F1), _ptr(self.F2), _ptr(self.G)
        h = ctypes.c_void_p()
        with torch.cuda.device(d):
            _lib.check(L.rbp_build_mpc(ctypes.byref(desc), _stream_handle(d), ctypes.byref(h)), "rbp_build_mpc")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            _lib.load().rbp_destroy_mpc(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self) -> MpcResult:
        d, n, N = self.device, self.n, self.N
        f = dict(dtype=torch.float64, device=d)
        return MpcResult(X=torch.empty((n, N + 1, 6), **f), U=torch.empty((n, N, 3), **f),
                         cost=torch.empty(n, **f), status=torch.empty(n, dtype=torch.int32, device=d),
                         kkt=torch.empty(n, **f), iters=torch.empty(n, dtype=torch.int32, device=d))

    def solve(self, x0: torch.Tensor, ref: torch.Tensor, planes: torch.Tensor, max_iters: int = 40,
              tol: float = 1e-15, out: Optional[MpcResult] = None) -> MpcResult:
        o = out or self.alloc()
        rc = _lib.load().rbp_mpc_solve(self._h, _ptr(x0), _ptr(ref), _ptr(planes), int(max_iters), float(tol),
                                       _ptr(o.X), _ptr(o.U), _ptr(o.cost), _ptr(o.status), _ptr(o.kkt),
                                       _ptr(o.iters), _stream_handle(self.device))
        _lib.check(rc, "rbp_mpc_solve")
        return o
