"""Seeded synthetic inputs for the batched segment-QP workloads.

This module only draws numbers: it holds none of the method's arithmetic (no
Bezier operators, no constraint lifting, no solver).  Both the FP64 CPU
oracle and the HIP path consume what it returns.

The paper (Sec. IV, Figs. 4-5) measures on its own MuJoCo scenes and on the
ARCHER robot, not on a public suite, and never states the reachable-polytope
matrices of Theorem 2.  The generators below are synthetic stand-ins with the
paper's shapes: about 50,000 candidate edges (Sec. IV-A) and a few hundred
box obstacles (Figs. 4-5).

Seeding: instance ``i`` of workload ``cfg`` draws from
``default_rng(SeedSequence(1000 + cfg, spawn_key=(0, i)))`` and the shared
environment (obstacles, polytopes) from ``spawn_key=(1,)``, so any subset of
a batch regenerates exactly.

Conventions shared with the consumers (documented in include/rbp.h):

* ``vec(P)`` is point-major: ``y[3*k + c]`` is coordinate ``c`` of control
  point ``k``.
* Reachable rows are stored in the literal form ``H vec(P) <= h0 + G x0``.
  They are drawn in the displacement frame ``H vec(P - 1 (x) P0) <= h0 + G' x0``
  (dynamics do not depend on where the segment starts) and stored with
  ``G = G' + H (1 (x) [I3 0])`` so the stored rows stay affine in ``x0``.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
import os
from typing import Dict, Optional, Sequence

import numpy as np

DIM = 3
T_DEFAULT = 1.0
VMAX = 3.0
AMAX = 5.0
# reachable-row offsets for the cluttered-environment batches: shifted from
# U[1,3] so that about 30% of the edges come out infeasible
H0_CLUTTER = (1.3, 3.3)
# offsets of a reachable block shared by all edges: with one block the
# feasible fraction follows the block, so it is shifted to leave about a
# third of the 50,000 edges infeasible, as in the per-edge batch
H0_SHARED = (1.6, 3.6)
# reachable-row offsets of the chain segments
H0_CHAIN = (2.0, 4.0)


def instance_rng(cfg: int, i: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(1000 + cfg, spawn_key=(0, int(i))))


def env_rng(cfg: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(1000 + cfg, spawn_key=(1,)))


@dataclass
class SegmentBatch:
    """A batch of segment problems in the layout the C ABI consumes.

    Shared polytope table: polytope ``j`` owns faces ``poly_off[j]:poly_off[j+1]``
    of ``A_face`` (F x 3) and ``b_face`` (F).  Instance ``i`` uses polytope
    ``poly_idx[i]``, has degree ``degree[i]`` and ``reach_off[i+1]-reach_off[i]``
    reachable rows whose dense coefficients sit in
    ``H[H_off[i]:H_off[i+1]]`` (row-major, ``3*(degree+1)`` columns), with
    ``h0``/``G`` rows at the same row offsets.
    """

    name: str
    degree: np.ndarray          # int32 [N]
    T: np.ndarray               # float64 [N]
    vmax: float
    amax: float
    poly_off: np.ndarray        # int32 [n_poly+1]
    A_face: np.ndarray          # float64 [F, 3]
    b_face: np.ndarray          # float64 [F]
    poly_idx: np.ndarray        # int32 [N]
    reach_off: np.ndarray       # int64 [N+1]
    H_off: np.ndarray           # int64 [N+1]
    H: np.ndarray               # float64 [sum r_i * 3(p_i+1)]
    h0: np.ndarray              # float64 [R]
    G: np.ndarray               # float64 [R, 6]
    x0: np.ndarray              # float64 [N, 6]
    goal: np.ndarray            # float64 [N, 3]
    meta: Dict[str, object] = field(default_factory=dict)
    # shared reachable blocks: None, or int32 [N] indexing blocks of
    # reach_off / H_off (which then have one entry per block, plus one)
    reach_idx: Optional[np.ndarray] = None
    # start velocity pinned as well as the start position (b'(0) = x0[3:6])
    pin_v0: bool = False

    @property
    def n(self) -> int:
        return int(self.degree.shape[0])

    def block(self, i: int) -> int:
        return int(i) if self.reach_idx is None else int(self.reach_idx[i])

    def reach_rows(self, i: int) -> int:
        k = self.block(i)
        return int(self.reach_off[k + 1] - self.reach_off[k])

    def instance(self, i: int) -> dict:
        """Plain per-instance view (numpy arrays, FP64)."""
        p = int(self.degree[i])
        j = int(self.poly_idx[i])
        f0, f1 = int(self.poly_off[j]), int(self.poly_off[j + 1])
        k = self.block(i)
        r0, r1 = int(self.reach_off[k]), int(self.reach_off[k + 1])
        h0_, h1_ = int(self.H_off[k]), int(self.H_off[k + 1])
        return dict(
            p=p, T=float(self.T[i]), vmax=float(self.vmax), amax=float(self.amax),
            A_face=self.A_face[f0:f1].copy(), b_face=self.b_face[f0:f1].copy(),
            H=self.H[h0_:h1_].reshape(r1 - r0, 3 * (p + 1)).copy(),
            h0=self.h0[r0:r1].copy(), G=self.G[r0:r1].copy(),
            x0=self.x0[i].copy(), goal=self.goal[i].copy(), pin_v0=bool(self.pin_v0),
        )

    def expanded(self) -> "SegmentBatch":
        """The same problems with every instance holding its own copy of its
        reachable block (the per-instance layout)."""
        if self.reach_idx is None:
            return self
        k = np.asarray(self.reach_idx, np.int64)
        r = (self.reach_off[k + 1] - self.reach_off[k])
        hsz = (self.H_off[k + 1] - self.H_off[k])
        reach_off = np.concatenate([[0], np.cumsum(r)]).astype(np.int64)
        H_off = np.concatenate([[0], np.cumsum(hsz)]).astype(np.int64)
        H = np.concatenate([self.H[self.H_off[b]:self.H_off[b + 1]] for b in k]) if len(k) else np.zeros(0)
        h0 = np.concatenate([self.h0[self.reach_off[b]:self.reach_off[b + 1]] for b in k]) if len(k) else np.zeros(0)
        G = np.concatenate([self.G[self.reach_off[b]:self.reach_off[b + 1]] for b in k]) if len(k) else np.zeros((0, 6))
        return dataclasses.replace(self, name=f"{self.name}[expanded]", reach_off=reach_off, H_off=H_off, H=H,
                                   h0=h0, G=G.reshape(-1, 6), reach_idx=None)

    def subset(self, idx: Sequence[int]) -> "SegmentBatch":
        idx = np.asarray(idx, dtype=np.int64)
        if self.reach_idx is not None:
            return dataclasses.replace(self, name=f"{self.name}[subset]", degree=self.degree[idx].copy(),
                                       T=self.T[idx].copy(), poly_idx=self.poly_idx[idx].copy(),
                                       x0=self.x0[idx].copy(), goal=self.goal[idx].copy(),
                                       reach_idx=self.reach_idx[idx].copy(),
                                       meta=dict(self.meta, subset=idx.tolist()[:16]))
        r = self.reach_off[idx + 1] - self.reach_off[idx]
        hsz = self.H_off[idx + 1] - self.H_off[idx]
        reach_off = np.zeros(len(idx) + 1, np.int64)
        reach_off[1:] = np.cumsum(r)
        H_off = np.zeros(len(idx) + 1, np.int64)
        H_off[1:] = np.cumsum(hsz)
        H = np.concatenate([self.H[self.H_off[i]:self.H_off[i + 1]] for i in idx]) if len(idx) else np.zeros(0)
        h0 = np.concatenate([self.h0[self.reach_off[i]:self.reach_off[i + 1]] for i in idx]) if len(idx) else np.zeros(0)
        G = np.concatenate([self.G[self.reach_off[i]:self.reach_off[i + 1]] for i in idx]) if len(idx) else np.zeros((0, 6))
        return SegmentBatch(
            name=f"{self.name}[subset]", degree=self.degree[idx].copy(), T=self.T[idx].copy(),
            vmax=self.vmax, amax=self.amax, poly_off=self.poly_off, A_face=self.A_face,
            b_face=self.b_face, poly_idx=self.poly_idx[idx].copy(), reach_off=reach_off,
            H_off=H_off, H=H, h0=h0, G=G.reshape(-1, 6), x0=self.x0[idx].copy(),
            goal=self.goal[idx].copy(), meta=dict(self.meta, subset=idx.tolist()[:16]), pin_v0=self.pin_v0,
        )


# ---------------------------------------------------------------------------
# building blocks (draws only)
# ---------------------------------------------------------------------------

def _reach_block(rng: np.random.Generator, r: int, p: int, h0_lo: float = 1.0, h0_hi: float = 3.0):
    """r reachable rows over 3(p+1) coefficients: unit-norm Gaussian rows,
    h0 ~ U[h0_lo, h0_hi], G' ~ N(0, 0.1^2); G returned in the literal
    (absolute) form."""
    ncol = 3 * (p + 1)
    H = rng.standard_normal((r, ncol))
    H /= np.linalg.norm(H, axis=1, keepdims=True)
    h0 = rng.uniform(h0_lo, h0_hi, size=r)
    Gp = rng.normal(0.0, 0.1, size=(r, 6))
    G = Gp.copy()
    # displacement frame -> literal frame: add H (1 (x) [I3 0]) to the x0 map
    G[:, :3] += H.reshape(r, p + 1, 3).sum(axis=1)
    return H, h0, G


def _box_polytope(rng: np.random.Generator, n_faces: int, centre: np.ndarray):
    """A bounded polytope containing ``centre``: 6 axis faces with half-widths
    U[0.5,2] plus ``n_faces-6`` Gaussian-normal cuts at offset n.c + U[0.5,2]."""
    w = rng.uniform(0.5, 2.0, size=3)
    A = np.concatenate([np.eye(3), -np.eye(3)])
    b = np.concatenate([centre + w, -(centre - w)])
    k = n_faces - 6
    if k > 0:
        nrm = rng.standard_normal((k, 3))
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        off = nrm @ centre + rng.uniform(0.5, 2.0, size=k)
        A = np.concatenate([A, nrm])
        b = np.concatenate([b, off])
    return A, b, w


def _inside(A: np.ndarray, b: np.ndarray, pts: np.ndarray) -> np.ndarray:
    return np.all(pts @ A.T <= b, axis=-1)


def _finalize(name, degree, T, poly_A, poly_b, poly_idx, Hs, h0s, Gs, x0, goal, meta, vmax=VMAX, amax=AMAX):
    poly_off = np.zeros(len(poly_A) + 1, np.int32)
    poly_off[1:] = np.cumsum([a.shape[0] for a in poly_A])
    reach_off = np.zeros(len(Hs) + 1, np.int64)
    reach_off[1:] = np.cumsum([h.shape[0] for h in Hs])
    H_off = np.zeros(len(Hs) + 1, np.int64)
    H_off[1:] = np.cumsum([h.size for h in Hs])
    return SegmentBatch(
        name=name, degree=np.asarray(degree, np.int32), T=np.asarray(T, np.float64),
        vmax=vmax, amax=amax, poly_off=poly_off,
        A_face=np.ascontiguousarray(np.concatenate(poly_A)),
        b_face=np.ascontiguousarray(np.concatenate(poly_b)),
        poly_idx=np.asarray(poly_idx, np.int32), reach_off=reach_off, H_off=H_off,
        H=np.ascontiguousarray(np.concatenate([h.ravel() for h in Hs])),
        h0=np.ascontiguousarray(np.concatenate(h0s)),
        G=np.ascontiguousarray(np.concatenate(Gs).reshape(-1, 6)),
        x0=np.ascontiguousarray(np.asarray(x0, np.float64).reshape(-1, 6)),
        goal=np.ascontiguousarray(np.asarray(goal, np.float64).reshape(-1, 3)), meta=meta,
    )


# ---------------------------------------------------------------------------
# workload 0: 64 independent degree-7 segments, each in its own axis box
# ---------------------------------------------------------------------------

def gen_cfg0(n: int = 64, indices: Optional[Sequence[int]] = None, p: int = 7, r: int = 32) -> SegmentBatch:
    idx = range(n) if indices is None else indices
    poly_A, poly_b, Hs, h0s, Gs, x0s, goals = [], [], [], [], [], [], []
    for i in idx:
        rng = instance_rng(0, i)
        c = rng.uniform(0.0, 10.0, size=3)
        w = rng.uniform(0.5, 2.0, size=3)
        pos0 = c + 0.9 * w * rng.uniform(-1.0, 1.0, size=3)
        g = c + 0.9 * w * rng.uniform(-1.0, 1.0, size=3)
        v0 = rng.uniform(-1.0, 1.0, size=3)
        H, h0, G = _reach_block(rng, r, p)
        poly_A.append(np.concatenate([np.eye(3), -np.eye(3)]))
        poly_b.append(np.concatenate([c + w, -(c - w)]))
        Hs.append(H); h0s.append(h0); Gs.append(G)
        x0s.append(np.concatenate([pos0, v0])); goals.append(g)
    m = len(x0s)
    return _finalize("seg64_p7_box", [p] * m, [T_DEFAULT] * m, poly_A, poly_b, np.arange(m),
                     Hs, h0s, Gs, x0s, goals, dict(cfg=0))


# ---------------------------------------------------------------------------
# cluttered environment shared by workloads 1, 2 and 4
# ---------------------------------------------------------------------------

@dataclass
class Environment:
    obs_lo: np.ndarray
    obs_hi: np.ndarray
    centres: np.ndarray
    halfw: np.ndarray
    poly_A: list
    poly_b: list
    knn: np.ndarray


def make_environment(cfg: int, n_obst: int = 200, n_poly: int = 2000, faces=(8, 24), k_nn: int = 4) -> Environment:
    rng = env_rng(cfg)
    oc = rng.uniform(0.0, 10.0, size=(n_obst, 3))
    osz = rng.uniform(0.2, 1.5, size=(n_obst, 3))
    lo, hi = oc - osz / 2, oc + osz / 2
    centres, halfw, pA, pb = [], [], [], []
    for _ in range(n_poly):
        while True:
            c = rng.uniform(0.0, 10.0, size=3)
            if not np.any(np.all((c >= lo) & (c <= hi), axis=1)):
                break
        nf = int(rng.integers(faces[0], faces[1] + 1))
        A, b, w = _box_polytope(rng, nf, c)
        centres.append(c); halfw.append(w); pA.append(A); pb.append(b)
    centres = np.asarray(centres)
    d2 = ((centres[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    knn = np.argsort(d2, axis=1)[:, :k_nn]
    return Environment(lo, hi, centres, np.asarray(halfw), pA, pb, knn)


_ENV_CACHE: Dict[tuple, Environment] = {}


def environment(cfg: int, **kw) -> Environment:
    key = (cfg, tuple(sorted(kw.items())))
    if key not in _ENV_CACHE:
        _ENV_CACHE[key] = make_environment(cfg, **kw)
    return _ENV_CACHE[key]


def _sample_in(rng, A, b, c, w, tries: int = 8, batch: int = 64):
    for _ in range(tries):
        cand = c + w * rng.uniform(-1.0, 1.0, size=(batch, 3))
        ok = _inside(A, b, cand)
        if ok.any():
            return cand[int(np.argmax(ok))]
    return c.copy()


def _edge(rng, env: Environment, p: int, r: int):
    j = int(rng.integers(0, len(env.poly_A)))
    A, b = env.poly_A[j], env.poly_b[j]
    c, w = env.centres[j], env.halfw[j]
    pos0 = _sample_in(rng, A, b, c, w)
    goal = None
    for nb in rng.permutation(env.knn[j]):
        An, bn = env.poly_A[nb], env.poly_b[nb]
        for _ in range(4):
            cand = c + w * rng.uniform(-1.0, 1.0, size=(256, 3))
            ok = _inside(A, b, cand) & _inside(An, bn, cand)
            if ok.any():
                goal = cand[int(np.argmax(ok))]
                break
        if goal is not None:
            break
    if goal is None:                       # no overlap with any near neighbour
        goal = _sample_in(rng, A, b, c, w)
    v0 = rng.uniform(-1.0, 1.0, size=3)
    H, h0, G = _reach_block(rng, r, p, *H0_CLUTTER)
    return j, np.concatenate([pos0, v0]), goal, H, h0, G


def gen_cfg1(n: int = 50_000, indices: Optional[Sequence[int]] = None, cfg: int = 1) -> SegmentBatch:
    """Edge-evaluation batch: degree-7 segments, start polytope from a shared
    table of 2,000 free-space polytopes (8-24 faces) placed among 200 box
    obstacles; the goal lies where the start polytope meets one of its 4
    nearest neighbours."""
    env = environment(cfg)
    idx = range(n) if indices is None else indices
    pidx, Hs, h0s, Gs, x0s, goals = [], [], [], [], [], []
    for i in idx:
        rng = instance_rng(cfg, i)
        j, x0, g, H, h0, G = _edge(rng, env, 7, 32)
        pidx.append(j); Hs.append(H); h0s.append(h0); Gs.append(G); x0s.append(x0); goals.append(g)
    m = len(x0s)
    return _finalize("edges50k_p7_clutter", [7] * m, [T_DEFAULT] * m, env.poly_A, env.poly_b, pidx,
                     Hs, h0s, Gs, x0s, goals, dict(cfg=cfg))


def gen_cfg2(n: int = 200_000, indices: Optional[Sequence[int]] = None) -> SegmentBatch:
    """Uneven sizes: degree U{3..9}, 6-40 faces per polytope, 16-128 reachable rows."""
    env = environment(2, faces=(6, 40))
    idx = range(n) if indices is None else indices
    deg, pidx, Hs, h0s, Gs, x0s, goals = [], [], [], [], [], [], []
    for i in idx:
        rng = instance_rng(2, i)
        p = int(rng.integers(3, 10))
        r = int(rng.integers(16, 129))
        j, x0, g, H, h0, G = _edge(rng, env, p, r)
        deg.append(p); pidx.append(j); Hs.append(H); h0s.append(h0); Gs.append(G); x0s.append(x0); goals.append(g)
    m = len(x0s)
    return _finalize("uneven200k_p3to9", deg, [T_DEFAULT] * m, env.poly_A, env.poly_b, pidx,
                     Hs, h0s, Gs, x0s, goals, dict(cfg=2))


def upstream_grads(cfg: int, n: int, ncol: int = 24, indices: Optional[Sequence[int]] = None) -> np.ndarray:
    """Upstream gradient on P* for the differentiation workload: N(0,1) per
    entry, seeded per instance (stream spawn_key=(2, i))."""
    idx = range(n) if indices is None else indices
    out = np.empty((len(idx), ncol))
    for k, i in enumerate(idx):
        rng = np.random.default_rng(np.random.SeedSequence(1000 + cfg, spawn_key=(2, int(i))))
        out[k] = rng.standard_normal(ncol)
    return out


GENERATORS = {0: gen_cfg0, 1: gen_cfg1, 2: gen_cfg2}


def concat(parts) -> SegmentBatch:
    """Join batches that share one polytope table (same workload)."""
    parts = [p for p in parts if p.n > 0] or list(parts)[:1]
    first = parts[0]
    assert all(p.reach_idx is None for p in parts), "concat joins per-instance reachable blocks only"
    reach = np.concatenate([[0]] + [np.diff(p.reach_off) for p in parts]).cumsum()
    hsz = np.concatenate([[0]] + [np.diff(p.H_off) for p in parts]).cumsum()
    return SegmentBatch(
        name=first.name, degree=np.concatenate([p.degree for p in parts]),
        T=np.concatenate([p.T for p in parts]), vmax=first.vmax, amax=first.amax,
        poly_off=first.poly_off, A_face=first.A_face, b_face=first.b_face,
        poly_idx=np.concatenate([p.poly_idx for p in parts]),
        reach_off=reach.astype(np.int64), H_off=hsz.astype(np.int64),
        H=np.concatenate([p.H for p in parts]), h0=np.concatenate([p.h0 for p in parts]),
        G=np.concatenate([p.G for p in parts]).reshape(-1, 6),
        x0=np.concatenate([p.x0 for p in parts]), goal=np.concatenate([p.goal for p in parts]),
        meta=dict(first.meta),
    )


def with_shared_reach(b: SegmentBatch, r: int = 32, h0_range=H0_SHARED, seed: int = 7) -> SegmentBatch:
    """The same edges with one reachable block per degree shared by every
    instance of that degree (the paper computes the reachable polytope once
    and uses it for all edges, Sec. III-A); block draws as for a single edge,
    from their own seed."""
    degrees = sorted(set(int(p) for p in b.degree))
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(3,)))
    Hs, h0s, Gs = [], [], []
    for p in degrees:
        H, h0, G = _reach_block(rng, r, p, *h0_range)
        Hs.append(H); h0s.append(h0); Gs.append(G)
    slot = {p: k for k, p in enumerate(degrees)}
    reach_idx = np.asarray([slot[int(p)] for p in b.degree], np.int32)
    reach_off = np.concatenate([[0], np.cumsum([h.shape[0] for h in Hs])]).astype(np.int64)
    H_off = np.concatenate([[0], np.cumsum([h.size for h in Hs])]).astype(np.int64)
    return dataclasses.replace(b, name=f"{b.name}_shared_reach", reach_off=reach_off, H_off=H_off,
                               H=np.concatenate([h.ravel() for h in Hs]), h0=np.concatenate(h0s),
                               G=np.concatenate(Gs).reshape(-1, 6), reach_idx=reach_idx,
                               meta=dict(b.meta, shared_reach=dict(r=r, h0=list(h0_range), seed=seed)))


def with_pinned_velocity(b: SegmentBatch) -> SegmentBatch:
    """The same edges with the start velocity pinned too (Lemma 1's
    full-state start: P_1 = P_0 + (T/p) vel(x0))."""
    return dataclasses.replace(b, name=f"{b.name}_pinned_v0", pin_v0=True, meta=dict(b.meta, pin_v0=True))


def _gen_chunk(args):
    cfg, idx = args
    if cfg == 0:
        return gen_cfg0(indices=idx)
    if cfg in (1, 4):
        return gen_cfg1(indices=idx, cfg=1)
    return gen_cfg2(indices=idx)


def generate(cfg: int, n: int, workers: Optional[int] = None) -> SegmentBatch:
    """Workload ``cfg`` with ``n`` instances, drawn in parallel processes.
    Every instance has its own seed, so the result equals the serial one."""
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or n < 2000:
        return _gen_chunk((cfg, list(range(n))))
    chunks = [list(c) for c in np.array_split(np.arange(n), workers * 4) if len(c)]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_gen_chunk, [(cfg, c) for c in chunks])
    out = concat(parts)
    out.name = parts[0].name
    return out


def from_instances(insts, name: str = "custom") -> SegmentBatch:
    """Pack per-instance dicts (the layout of ``SegmentBatch.instance``) into
    a batch; each instance gets its own polytope."""
    pins = {bool(d.get("pin_v0", False)) for d in insts}
    assert len(pins) <= 1, "pin_v0 is a property of the whole batch"
    if pins == {True}:
        return dataclasses.replace(from_instances([dict(d, pin_v0=False) for d in insts], name), pin_v0=True)
    return _finalize(name, [d["p"] for d in insts], [d["T"] for d in insts],
                     [np.asarray(d["A_face"], float) for d in insts],
                     [np.asarray(d["b_face"], float) for d in insts], np.arange(len(insts)),
                     [np.asarray(d["H"], float).reshape(-1, 3 * (d["p"] + 1)) for d in insts],
                     [np.asarray(d["h0"], float) for d in insts],
                     [np.asarray(d["G"], float).reshape(-1, 6) for d in insts],
                     [np.asarray(d["x0"], float) for d in insts],
                     [np.asarray(d["goal"], float) for d in insts], dict(cfg=-1),
                     vmax=insts[0]["vmax"], amax=insts[0]["amax"]) if insts else _empty(name)


def _empty(name):
    return SegmentBatch(name=name, degree=np.zeros(0, np.int32), T=np.zeros(0), vmax=VMAX, amax=AMAX,
                        poly_off=np.zeros(2, np.int32) + np.array([0, 6], np.int32),
                        A_face=np.concatenate([np.eye(3), -np.eye(3)]), b_face=np.ones(6),
                        poly_idx=np.zeros(0, np.int32), reach_off=np.zeros(1, np.int64),
                        H_off=np.zeros(1, np.int64), H=np.zeros(0), h0=np.zeros(0), G=np.zeros((0, 6)),
                        x0=np.zeros((0, 6)), goal=np.zeros((0, 3)))


# ---------------------------------------------------------------------------
# workload 3: multi-segment chains through a corridor of overlapping polytopes
# ---------------------------------------------------------------------------

@dataclass
class ChainBatch:
    """N chains; chain c has segments seg_off[c]..seg_off[c+1]-1.  Segment s
    uses polytope poly_idx[s] of the shared table and reachable rows
    reach_off[s]..reach_off[s+1]-1 (coefficients at H_off[s], 3(p+1) columns)."""

    name: str
    degree: int
    T: float
    vmax: float
    amax: float
    seg_off: np.ndarray        # int64 [N+1]
    poly_off: np.ndarray       # int32 [n_poly+1]
    A_face: np.ndarray         # [F,3]
    b_face: np.ndarray         # [F]
    poly_idx: np.ndarray       # int32 [n_seg]
    reach_off: np.ndarray      # int64 [n_seg+1]
    H_off: np.ndarray          # int64 [n_seg+1]
    H: np.ndarray
    h0: np.ndarray
    G: np.ndarray              # [R, 6]
    x0: np.ndarray             # [N, 6] start state of the chain
    goal: np.ndarray           # [N, 3]

    @property
    def n(self) -> int:
        return int(self.seg_off.shape[0] - 1)

    def chain(self, c: int) -> dict:
        s0, s1 = int(self.seg_off[c]), int(self.seg_off[c + 1])
        p = self.degree
        segs = []
        for s in range(s0, s1):
            j = int(self.poly_idx[s])
            f0, f1 = int(self.poly_off[j]), int(self.poly_off[j + 1])
            r0, r1 = int(self.reach_off[s]), int(self.reach_off[s + 1])
            segs.append(dict(A_face=self.A_face[f0:f1].copy(), b_face=self.b_face[f0:f1].copy(),
                             H=self.H[self.H_off[s]:self.H_off[s + 1]].reshape(r1 - r0, 3 * (p + 1)).copy(),
                             h0=self.h0[r0:r1].copy(), G=self.G[r0:r1].copy()))
        return dict(p=p, T=self.T, vmax=self.vmax, amax=self.amax, x0=self.x0[c].copy(),
                    goal=self.goal[c].copy(), segments=segs)


def _overlap_point(rng, A1, b1, c1, w1, A2, b2, tries=6):
    for _ in range(tries):
        cand = c1 + w1 * rng.uniform(-1.0, 1.0, size=(256, 3))
        ok = _inside(A1, b1, cand) & _inside(A2, b2, cand)
        if ok.any():
            return cand[int(np.argmax(ok))]
    return None


def gen_cfg3(n: int = 8192, indices: Optional[Sequence[int]] = None, p: int = 7, r: int = 32) -> ChainBatch:
    """Chains of S ~ U{4..12} degree-7 segments; polytope centres follow a
    random walk with steps U[0.8, 1.5] m (a step is redrawn until consecutive
    polytopes overlap); start inside the first polytope, goal inside the last."""
    idx = range(n) if indices is None else indices
    seg_off = [0]
    polys_A, polys_b, pidx, Hs, h0s, Gs, x0s, goals = [], [], [], [], [], [], [], []
    for i in idx:
        rng = instance_rng(3, i)
        S = int(rng.integers(4, 13))
        c = rng.uniform(2.0, 8.0, size=3)
        nf = int(rng.integers(8, 25))
        A, b, w = _box_polytope(rng, nf, c)
        chain = [(A, b, c, w)]
        while len(chain) < S:
            for _ in range(50):
                d = rng.standard_normal(3)
                d *= rng.uniform(0.8, 1.5) / np.linalg.norm(d)
                c2 = chain[-1][2] + d
                nf2 = int(rng.integers(8, 25))
                A2, b2, w2 = _box_polytope(rng, nf2, c2)
                if _overlap_point(rng, chain[-1][0], chain[-1][1], chain[-1][2], chain[-1][3], A2, b2) is not None:
                    chain.append((A2, b2, c2, w2))
                    break
            else:
                raise RuntimeError("corridor step not found")
        start = _sample_in(rng, chain[0][0], chain[0][1], chain[0][2], chain[0][3])
        goal = _sample_in(rng, chain[-1][0], chain[-1][1], chain[-1][2], chain[-1][3])
        v0 = rng.uniform(-1.0, 1.0, size=3)
        for (A_, b_, _, _) in chain:
            pidx.append(len(polys_A))
            polys_A.append(A_); polys_b.append(b_)
            H, h0, G = _reach_block(rng, r, p, *H0_CHAIN)
            Hs.append(H); h0s.append(h0); Gs.append(G)
        seg_off.append(seg_off[-1] + S)
        x0s.append(np.concatenate([start, v0])); goals.append(goal)
    poly_off = np.zeros(len(polys_A) + 1, np.int32)
    poly_off[1:] = np.cumsum([a.shape[0] for a in polys_A])
    reach_off = np.zeros(len(Hs) + 1, np.int64)
    reach_off[1:] = np.cumsum([h.shape[0] for h in Hs])
    H_off = np.zeros(len(Hs) + 1, np.int64)
    H_off[1:] = np.cumsum([h.size for h in Hs])
    return ChainBatch(name="chains8k_p7", degree=p, T=T_DEFAULT, vmax=VMAX, amax=AMAX,
                      seg_off=np.asarray(seg_off, np.int64), poly_off=poly_off,
                      A_face=np.concatenate(polys_A), b_face=np.concatenate(polys_b),
                      poly_idx=np.asarray(pidx, np.int32), reach_off=reach_off, H_off=H_off,
                      H=np.concatenate([h.ravel() for h in Hs]), h0=np.concatenate(h0s),
                      G=np.concatenate(Gs).reshape(-1, 6), x0=np.asarray(x0s).reshape(-1, 6),
                      goal=np.asarray(goals).reshape(-1, 3))


def concat_chains(parts) -> ChainBatch:
    """Join path batches (each part has its own polytopes)."""
    first = parts[0]
    seg_off, poly_off, pidx, reach_off, H_off = [np.zeros(1, np.int64)], [np.zeros(1, np.int64)], [], \
        [np.zeros(1, np.int64)], [np.zeros(1, np.int64)]
    npoly = nseg = nf_tot = nr_tot = nh_tot = 0
    for pt in parts:
        seg_off.append(pt.seg_off[1:] + nseg)
        poly_off.append(pt.poly_off[1:].astype(np.int64) + nf_tot)
        pidx.append(pt.poly_idx.astype(np.int64) + npoly)
        reach_off.append(pt.reach_off[1:] + nr_tot)
        H_off.append(pt.H_off[1:] + nh_tot)
        nseg += int(pt.seg_off[-1]); npoly += len(pt.poly_off) - 1
        nf_tot += int(pt.poly_off[-1]); nr_tot += int(pt.reach_off[-1]); nh_tot += int(pt.H_off[-1])
    return ChainBatch(
        name=first.name, degree=first.degree, T=first.T, vmax=first.vmax, amax=first.amax,
        seg_off=np.concatenate(seg_off), poly_off=np.concatenate(poly_off).astype(np.int32),
        A_face=np.concatenate([p.A_face for p in parts]), b_face=np.concatenate([p.b_face for p in parts]),
        poly_idx=np.concatenate(pidx).astype(np.int32), reach_off=np.concatenate(reach_off),
        H_off=np.concatenate(H_off), H=np.concatenate([p.H for p in parts]),
        h0=np.concatenate([p.h0 for p in parts]), G=np.concatenate([p.G for p in parts]).reshape(-1, 6),
        x0=np.concatenate([p.x0 for p in parts]), goal=np.concatenate([p.goal for p in parts]))


def _gen_chain_chunk(idx):
    return gen_cfg3(indices=idx)


def generate_chains(n: int = 8192, workers: Optional[int] = None) -> ChainBatch:
    """The path workload drawn in parallel processes (equal to the serial draw)."""
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or n < 256:
        return gen_cfg3(indices=list(range(n)))
    chunks = [list(c) for c in np.array_split(np.arange(n), workers * 4) if len(c)]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_gen_chain_chunk, chunks)
    return concat_chains(parts)


# ---------------------------------------------------------------------------
# Cutting graph edges against obstacles (Sec. III-B, Alg. 2, eq. Cut-QP)
# ---------------------------------------------------------------------------
@dataclass
class CutBatch:
    """Edges (degree-p Bezier control points) and obstacles: axis-aligned
    boxes, then convex polytopes {x : A x <= b}.

    P[e, k, c]: coordinate c of control point k of edge e; box_lo/box_hi:
    [n_boxes, 3]; polytope j owns rows pob_off[j] .. pob_off[j+1]-1 of
    pob_A [rows, 3] and pob_b [rows].  Obstacle o < n_boxes is box o, obstacle
    n_boxes + j is polytope j."""
    name: str
    degree: int
    P: np.ndarray
    box_lo: np.ndarray
    box_hi: np.ndarray
    pob_off: np.ndarray = field(default_factory=lambda: np.zeros(1, np.int32))
    pob_A: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    pob_b: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def n_edges(self) -> int:
        return self.P.shape[0]

    @property
    def n_boxes(self) -> int:
        return self.box_lo.shape[0]

    @property
    def n_polytopes(self) -> int:
        return len(self.pob_off) - 1

    @property
    def n_obstacles(self) -> int:
        return self.n_boxes + self.n_polytopes

    def polytope(self, j: int):
        a, z = self.pob_off[j], self.pob_off[j + 1]
        return self.pob_A[a:z], self.pob_b[a:z]


def polytope_obstacles(n: int, rng: np.random.Generator, extent: float = 10.0):
    """Convex polytope obstacles: centre c uniform in [0, extent]^3, the six
    axis faces at half-widths U[0.1, 0.75] plus 2-10 cuts with unit Gaussian
    normals at offset n.c + U[0.1, 0.75] (bounded, centre inside; sizes like
    the box obstacles').  Returns (row offsets, A, b)."""
    off, As, bs = [0], [], []
    for _ in range(n):
        c = rng.uniform(0.0, extent, 3)
        w = rng.uniform(0.1, 0.75, 3)
        k = int(rng.integers(2, 11))
        N = rng.standard_normal((k, 3))
        N /= np.linalg.norm(N, axis=1, keepdims=True)
        A = np.concatenate([np.eye(3), -np.eye(3), N])
        b = np.concatenate([c + w, -(c - w), N @ c + rng.uniform(0.1, 0.75, k)])
        As.append(A); bs.append(b); off.append(off[-1] + A.shape[0])
    return (np.asarray(off, np.int32), np.ascontiguousarray(np.concatenate(As)) if As else np.zeros((0, 3)),
            np.ascontiguousarray(np.concatenate(bs)) if bs else np.zeros(0))


def gen_cut(n_nodes: int = 5000, k_nn: int = 10, n_obst: int = 200, p: int = 7, cfg: int = 5,
            bend: float = 0.15, n_poly: int = 0) -> CutBatch:
    """Graph edges over the obstacle field of the cluttered environment: nodes
    uniform in [0, 10]^3 outside every obstacle, each joined to its k nearest
    neighbours (about n_nodes * k_nn edges; 5,000 nodes and 10 neighbours give
    the 50,000 edges of Sec. IV-A), the curve of an edge being the straight
    degree-p segment between its nodes with the interior control points moved
    by N(0, bend * length) per coordinate (curved edges).  Obstacles: the
    first n_obst boxes of the environment, then n_poly convex polytopes
    (``polytope_obstacles``, their own seed stream)."""
    env = environment(1)
    lo, hi = env.obs_lo[:n_obst], env.obs_hi[:n_obst]
    rng = np.random.default_rng(np.random.SeedSequence(1000 + cfg, spawn_key=(3,)))
    pob_off, pob_A, pob_b = polytope_obstacles(
        n_poly, np.random.default_rng(np.random.SeedSequence(1000 + cfg, spawn_key=(6,))))
    nodes = []
    while len(nodes) < n_nodes:
        c = rng.uniform(0.0, 10.0, size=(2 * n_nodes, 3))
        ok = ~np.any(np.all((c[:, None, :] >= lo[None]) & (c[:, None, :] <= hi[None]), axis=2), axis=1)
        for j in range(n_poly):
            Aj, bj = pob_A[pob_off[j]:pob_off[j + 1]], pob_b[pob_off[j]:pob_off[j + 1]]
            ok &= ~np.all(c @ Aj.T <= bj, axis=1)
        nodes.extend(c[ok][: n_nodes - len(nodes)])
    V = np.asarray(nodes)
    d2 = ((V[:, None, :] - V[None, :, :]) ** 2).sum(-1)
    np.fill_diagonal(d2, np.inf)
    nbr = np.argsort(d2, axis=1)[:, :k_nn]
    src = np.repeat(np.arange(n_nodes), k_nn)
    dst = nbr.reshape(-1)
    a, b = V[src], V[dst]
    t = np.arange(p + 1) / p
    P = a[:, None, :] + t[None, :, None] * (b - a)[:, None, :]
    length = np.linalg.norm(b - a, axis=1)
    P[:, 1:p, :] += rng.standard_normal((len(src), p - 1, 3)) * (bend * length)[:, None, None]
    return CutBatch(name=f"cut{len(src)}_o{n_obst}" + (f"_p{n_poly}" if n_poly else ""), degree=p,
                    P=np.ascontiguousarray(P), box_lo=np.ascontiguousarray(lo), box_hi=np.ascontiguousarray(hi),
                    pob_off=pob_off, pob_A=pob_A, pob_b=pob_b)


# ---------------------------------------------------------------------------
# Building the graph (Sec. III-A, Thm. 2) and adjacent hyperplanes (Alg. 2)
# ---------------------------------------------------------------------------
@dataclass
class GraphBatch:
    """Nodes V [n, d] and the reachable-polytope pair of Theorem 2 split into
    the columns on the start node (F1 [m, d]) and on the end node (F2 [m, d]),
    with G [m]: edge i -> j when F1 v_i + F2 v_j <= G."""
    name: str
    V: np.ndarray
    F1: np.ndarray
    F2: np.ndarray
    G: np.ndarray
    box_lo: np.ndarray
    box_hi: np.ndarray


def morton_order(P: np.ndarray, bits: int = 10) -> np.ndarray:
    """Indices sorting points of [0, 10]^3 along the Z-order curve."""
    q = np.clip((P / 10.0 * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(len(P), dtype=np.int64)
    for b in range(bits):
        for c in range(3):
            code |= ((q[:, c] >> b) & 1) << (3 * b + c)
    return np.argsort(code, kind="stable")


def gen_graph(n_nodes: int = 5000, m: int = 64, cfg: int = 6, n_obst: int = 200) -> GraphBatch:
    """Nodes uniform in [0, 10]^3 (the state space of interest), numbered
    along the Z-order curve; the reachable polytope has m rows on the
    displacement, a_k . (v_j - v_i) <= g_k with unit a_k uniform on the
    sphere and g_k ~ U[0.85, 1.1] (about 10 edges per node, the paper's
    5,000 nodes and 50,000 edges of Sec. IV-A), with F2 = A + N(0, 0.02^2) so
    the test is not purely translation invariant.  Obstacles: the first
    n_obst boxes of the environment (for the adjacent hyperplanes)."""
    rng = np.random.default_rng(np.random.SeedSequence(1000 + cfg, spawn_key=(4,)))
    V = rng.uniform(0.0, 10.0, size=(n_nodes, 3))
    V = np.ascontiguousarray(V[morton_order(V)])
    A = rng.standard_normal((m, 3))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    g = rng.uniform(0.85, 1.1, size=m)
    F2 = A + 0.02 * rng.standard_normal((m, 3))
    env = environment(1)
    return GraphBatch(name=f"graph{n_nodes}_m{m}", V=V, F1=np.ascontiguousarray(-A), F2=np.ascontiguousarray(F2),
                      G=g, box_lo=np.ascontiguousarray(env.obs_lo[:n_obst]),
                      box_hi=np.ascontiguousarray(env.obs_hi[:n_obst]))


# ---------------------------------------------------------------------------
# MPC refinement batches (eq. MPC, Sec. III-D)
# ---------------------------------------------------------------------------

@dataclass
class MpcBatch:
    """Independent MPC refinement problems over one horizon of N steps.

    Shared: step dt, tracking weight Q [6, 6], input weight R [3, 3],
    path-length weight w, and the reachable-polytope rows between
    consecutive nodes F1 x_k + F2 x_{k+1} <= G (F1, F2 [m, 6], G [m]).
    Per instance: start state x0 [6], reference states ref [N+1, 6] (the
    graph path sampled at dt), one separating plane per step
    planes [N, 4] = (n, l) with unit n (the segment from x_k to x_{k+1} must
    stay in n . y >= l), and the reference curve's acceleration at the nodes
    ref_u [N, 3]."""
    name: str
    N: int
    dt: float
    Q: np.ndarray
    R: np.ndarray
    w: float
    F1: np.ndarray
    F2: np.ndarray
    G: np.ndarray
    x0: np.ndarray
    ref: np.ndarray
    planes: np.ndarray
    ref_u: np.ndarray
    meta: Dict[str, object] = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x0.shape[0])

    def instance(self, i: int) -> dict:
        return dict(N=self.N, dt=self.dt, Q=self.Q, R=self.R, w=self.w, F1=self.F1, F2=self.F2, G=self.G,
                    x0=self.x0[i].copy(), ref=self.ref[i].copy(), planes=self.planes[i].copy())

    def subset(self, idx) -> "MpcBatch":
        idx = np.asarray(idx, np.int64)
        return dataclasses.replace(self, name=f"{self.name}[subset]", x0=self.x0[idx].copy(),
                                   ref=self.ref[idx].copy(), planes=self.planes[idx].copy(),
                                   ref_u=self.ref_u[idx].copy())


MPC_VMAX = 2.0
MPC_AMAX = 4.0


def mpc_reach_rows(dt: float, m_extra: int = 4, rng=None):
    """Rows on [x_k; x_{k+1}] (x = position, velocity): a velocity box on the
    next node, an input box |v_{k+1} - v_k| <= amax dt, and m_extra rows
    a . (v_{k+1} - v_k) <= g with unit a and g ~ U[0.05, 0.09] (acceleration
    limits of 0.5-0.9 m/s^2 in a few directions, below what the reference
    sometimes uses, so these rows become active; m = 12 + m_extra)."""
    rng = rng or np.random.default_rng(np.random.SeedSequence(1000 + 7, spawn_key=(5,)))
    rows1, rows2, rhs = [], [], []
    for c in range(3):
        for sgn in (1.0, -1.0):
            a1 = np.zeros(6); a2 = np.zeros(6); a2[3 + c] = sgn
            rows1.append(a1); rows2.append(a2); rhs.append(MPC_VMAX)
    for c in range(3):
        for sgn in (1.0, -1.0):
            a1 = np.zeros(6); a2 = np.zeros(6); a1[3 + c] = -sgn; a2[3 + c] = sgn
            rows1.append(a1); rows2.append(a2); rhs.append(MPC_AMAX * dt)
    for _ in range(m_extra):
        a = rng.standard_normal(3); a /= np.linalg.norm(a)
        a1 = np.zeros(6); a2 = np.zeros(6); a1[3:] = -a; a2[3:] = a
        rows1.append(a1); rows2.append(a2); rhs.append(rng.uniform(0.05, 0.09))
    return np.array(rows1), np.array(rows2), np.array(rhs)


def gen_mpc(n: int = 4096, N: int = 50, dt: float = 0.1, m_extra: int = 4, seed_cfg: int = 7,
            indices: Optional[Sequence[int]] = None) -> MpcBatch:
    """The paper's refinement setting (Sec. IV): a 50-node horizon at 0.1 s,
    path-length weight well above the tracking weight.  The reference samples
    a smooth curve whose acceleration is a(t) = sum of two sinusoids per axis
    (amplitude <= 0.5 each, frequency 1.5-3 rad/s, so |v| < vmax and
    |a| < amax), integrated in closed form; the start state is ref[0]
    plus a tracking error (position +-0.05, velocity +-0.1).  Plane k lies on
    the inner side of the reference's turn at node k (normal along minus the
    reference acceleration's component across the velocity, plus noise), at
    a distance U[0.05, 0.25] from the reference node (U[0.22, 0.5] for the
    first step, whose start is fixed), so cutting the corner, which the
    path-length weight (50, against 1 for position tracking) asks for, meets
    some of the planes."""
    idx = range(n) if indices is None else indices
    F1, F2, G = mpc_reach_rows(dt, m_extra)
    Q = np.diag([1.0, 1.0, 1.0, 0.1, 0.1, 0.1])
    R = 0.01 * np.eye(3)
    w = 50.0
    x0s, refs, planes, us = [], [], [], []
    t = dt * np.arange(N)
    for i in idx:
        rng = np.random.default_rng(np.random.SeedSequence(1000 + seed_cfg, spawn_key=(0, int(i))))
        amp = rng.uniform(0.2, 0.5, size=(2, 3))
        om = rng.uniform(1.5, 3.0, size=(2, 3))
        ph = rng.uniform(0, 2 * np.pi, size=(2, 3))
        p0 = rng.uniform(2.0, 8.0, 3)
        v0 = rng.uniform(-0.5, 0.5, 3)
        # the continuous curve with acceleration a(t), sampled at k dt
        tt = dt * np.arange(N + 1)[:, None]
        x = np.zeros((N + 1, 6))
        x[:, :3] = p0 + v0 * tt
        x[:, 3:] = v0
        for j in range(2):
            A_, w_, f_ = amp[j], om[j], ph[j]
            x[:, 3:] += A_ / w_ * (np.cos(f_) - np.cos(w_ * tt + f_))
            x[:, :3] += A_ / w_ * (tt * np.cos(f_) - (np.sin(w_ * tt + f_) - np.sin(f_)) / w_)
        u = (amp[0] * np.sin(om[0] * t[:, None] + ph[0]) + amp[1] * np.sin(om[1] * t[:, None] + ph[1]))
        pl = np.zeros((N, 4))
        for k in range(N):
            v = x[k, 3:]
            a = u[k]
            vv = v @ v
            side = a - (a @ v) / vv * v if vv > 1e-12 else a
            nrm = -side / max(np.linalg.norm(side), 1e-12) + 0.3 * rng.standard_normal(3)
            nrm /= np.linalg.norm(nrm)
            pl[k, :3] = nrm
            pl[k, 3] = nrm @ x[k, :3] - (rng.uniform(0.22, 0.5) if k == 0 else rng.uniform(0.05, 0.25))
        x0 = x[0].copy()
        x0[:3] += rng.uniform(-0.05, 0.05, 3)
        x0[3:] += rng.uniform(-0.1, 0.1, 3)
        x0s.append(x0); refs.append(x); planes.append(pl); us.append(u)
    return MpcBatch(name=f"mpc{len(x0s)}_n{N}", N=N, dt=dt, Q=Q, R=R, w=w, F1=F1, F2=F2, G=G,
                    x0=np.asarray(x0s).reshape(-1, 6), ref=np.asarray(refs).reshape(-1, N + 1, 6),
                    planes=np.asarray(planes).reshape(-1, N, 4), ref_u=np.asarray(us).reshape(-1, N, 3),
                    meta=dict(seed_cfg=seed_cfg, m=12 + m_extra))
