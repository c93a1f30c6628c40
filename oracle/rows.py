"""Dense FP64 constraint rows of one segment problem (oracle side).

Variable: ``y = vec(P)``, point-major, ``(p+1)*3`` entries.

* objective ``f(y) = y^T Q y = int_0^T |b''(t)|^2 dt`` (closed-form Bernstein
  Hessian, see ``bezier.hessian``);
* free-space faces: every control point satisfies ``A_f P_k <= b_f``, i.e.
  ``(I_{p+1} (x) A_f) y <= 1 (x) b_f``; by the convex-hull property
  (Property 1) the whole curve then stays in the polytope;
* velocity bounds on the derivative control points ``(p/T) Delta P_k``,
  componentwise, both signs;
* acceleration bounds on ``p(p-1)/T^2 Delta^2 P_k``, componentwise, both signs;
* reachable Bezier polytope (Theorem 2, stored affine in the start state):
  ``H y <= h0 + G x0``;
* equalities: ``P_0 = pos(x0)`` and ``P_p = goal`` (the edge joins the two
  waypoints, Sec. II-B graph semantics); with ``pin_v0`` also the start
  velocity, ``b'(0) = (p/T)(P_1 - P_0) = vel(x0)`` (the full-state start of
  Lemma 1: the derivative of a Bezier curve at t = 0 is p/T times its first
  control-polygon edge).

Inequalities are one-sided ``A y <= u``; each row carries a label
``(kind, k, j)`` used to map multipliers back to parameters.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bezier

FACE, VEL, ACC, REACH = 0, 1, 2, 3
KIND_NAMES = {FACE: "face", VEL: "vel", ACC: "acc", REACH: "reach"}


@dataclass
class SegmentQP:
    p: int
    T: float
    Q: np.ndarray        # n x n, f = y^T Q y
    A: np.ndarray        # m x n
    u: np.ndarray        # m
    E: np.ndarray        # 6 x n
    e: np.ndarray        # 6
    kind: np.ndarray     # m   row kind
    kidx: np.ndarray     # m   control point / difference index
    jidx: np.ndarray     # m   face index / coordinate / reach row
    # parameter Jacobians of the right-hand sides (for gradients)
    du_dx0: np.ndarray   # m x 6
    du_db: np.ndarray    # m x n_f
    de_dx0: np.ndarray   # 6 x 6
    de_dg: np.ndarray    # 6 x 3

    @property
    def n(self) -> int:
        return self.Q.shape[0]

    @property
    def m(self) -> int:
        return self.A.shape[0]


def build(inst: dict) -> SegmentQP:
    """Assemble the rows of one instance given as the plain dict of
    ``SegmentBatch.instance``."""
    p, T = inst["p"], inst["T"]
    vmax, amax = inst["vmax"], inst["amax"]
    Af, bf = inst["A_face"], inst["b_face"]
    H, h0, G = inst["H"], inst["h0"], inst["G"]
    x0, g = inst["x0"], inst["goal"]
    nf = Af.shape[0]
    npts = p + 1
    n = 3 * npts
    I3 = np.eye(3)

    blocks, rhs, kinds, ks, js, dx0, db = [], [], [], [], [], [], []

    # faces on every control point
    for k in range(npts):
        R = np.zeros((nf, n))
        R[:, 3 * k:3 * k + 3] = Af
        blocks.append(R); rhs.append(bf.copy())
        kinds += [FACE] * nf; ks += [k] * nf; js += list(range(nf))
        dx0.append(np.zeros((nf, 6)))
        db.append(np.eye(nf))

    # velocity and acceleration (both signs)
    for kind, order, bound in ((VEL, 1, vmax), (ACC, 2, amax)):
        scale = 1.0
        for q in range(order):
            scale *= (p - q)
        D = scale / T ** order * np.kron(bezier.diff_matrix(p, order), I3)
        nd = D.shape[0]
        for sgn in (1.0, -1.0):
            blocks.append(sgn * D); rhs.append(np.full(nd, bound))
            kinds += [kind] * nd
            ks += [r // 3 for r in range(nd)]
            js += [(r % 3) if sgn > 0 else 3 + (r % 3) for r in range(nd)]
            dx0.append(np.zeros((nd, 6))); db.append(np.zeros((nd, nf)))

    # reachable polytope
    r = H.shape[0]
    blocks.append(H.copy()); rhs.append(h0 + G @ x0)
    kinds += [REACH] * r; ks += [0] * r; js += list(range(r))
    dx0.append(G.copy()); db.append(np.zeros((r, nf)))

    A = np.concatenate(blocks)
    u = np.concatenate(rhs)

    pin_v0 = bool(inst.get("pin_v0", False))
    ne = 9 if pin_v0 else 6
    E = np.zeros((ne, n))
    E[0:3, 0:3] = I3
    E[3:6, 3 * p:3 * p + 3] = I3
    e = np.concatenate([x0[:3], g])
    de_dx0 = np.zeros((ne, 6)); de_dx0[0:3, 0:3] = I3
    de_dg = np.zeros((ne, 3)); de_dg[3:6, :] = I3
    if pin_v0:
        E[6:9, 3:6] = (p / T) * I3
        E[6:9, 0:3] = -(p / T) * I3
        e = np.concatenate([e, x0[3:6]])
        de_dx0[6:9, 3:6] = I3

    return SegmentQP(p=p, T=T, Q=bezier.hessian(p, T), A=A, u=u, E=E, e=e,
                     kind=np.asarray(kinds), kidx=np.asarray(ks), jidx=np.asarray(js),
                     du_dx0=np.concatenate(dx0), du_db=np.concatenate(db),
                     de_dx0=de_dx0, de_dg=de_dg)


def row_counts(qp: SegmentQP) -> dict:
    return {KIND_NAMES[k]: int((qp.kind == k).sum()) for k in (FACE, VEL, ACC, REACH)}
