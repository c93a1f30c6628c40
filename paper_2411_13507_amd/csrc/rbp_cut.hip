// Cutting graph edges against convex obstacles (Sec. III-B, Alg. 2, eq. Cut-QP;
// Assumption 1): axis-aligned boxes lo <= x <= hi and convex polytopes
// {x : A x <= b}.
//
// A pair is an edge (control points P_0..P_p of its Bezier curve) and an
// obstacle O.  By the convex-hull property (Property 1) the curve is free of
// O when conv(P) and O are disjoint.  Alg. 2 decides this in three steps:
//   1. a control point inside O                  -> 0 (may collide);
//   2. the supporting plane of O with normal n = centroid - (point of O
//      nearest the centroid) has every control point strictly beyond it
//                                                -> 1 (free);
//   3. otherwise the Cut-QP: |delta*|^2 > 0       -> 1, else 0.
// The Cut-QP's optimum is min over conv(P) of |(A x - b)_+|^2: for a box
// (unit rows) the squared distance between conv(P) and the box.  Step 3
// decides by the distance between conv(P) and O, computed with the
// Gilbert-Johnson-Keerthi iteration on the Minkowski difference (support
// points in closed form for a box, over the vertex table for a polytope),
// in FP64; the distance is zero exactly when the Cut-QP optimum is.  For a
// polytope the optimum itself is then computed, when asked for, by a second
// pass with one wavefront per pair (Newton steps over the pieces of the
// objective, each piece minimised exactly; see cut_value_kernel).
//
// Work split: steps 1-2 run for every pair, one thread per (edge, chunk of
// obstacles), control points in registers and the current obstacle read
// with uniform (scalar) loads; codes are written obstacle-major so a
// wavefront's stores are contiguous.  For a box the nearest point is a clamp
// and the supporting plane's offset a corner; for a polytope both come from
// its vertices (a GJK projection of the centroid, a maximum over the
// vertices).  Pairs left undecided (a fraction of a percent on cluttered
// graphs) are appended to a list with one atomic per wavefront, and a
// grid-stride kernel runs step 3 on the list.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "rbp_internal.hpp"
#include "rbp_wave.hpp"

namespace rbp {
namespace {

constexpr int kCutBlock = 256;
constexpr int kWave = 64;
constexpr int kObsChunk = 16;

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 axpy(double t, V3 a, V3 b) { return {b.x + t * a.x, b.y + t * a.y, b.z + t * a.z}; }

__global__ void cut_zero_kernel(unsigned long long* counter, int32_t* n_collide, int n_edges) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *counter = 0ull;
  if (i < n_edges) n_collide[i] = 0;
}

// Steps 1 and 2 of Alg. 2 for the pairs (e, o), o in this thread's chunk:
// boxes (kPoly = false, obstacles 0 .. n_box-1) or polytopes (kPoly = true,
// obstacles n_box .. n_obst-1), in separate launches so that the box kernel
// keeps its small register footprint.
template <int P, bool kPoly>
__global__ __launch_bounds__(kCutBlock) void cut_prefilter_kernel(CutArgs A) {
  constexpr int NP = P + 1;
  const int e = blockIdx.x * kCutBlock + threadIdx.x;
  const int o_first = kPoly ? A.n_box : 0, o_last = kPoly ? A.n_obst : A.n_box;
  const int o_begin = o_first + blockIdx.y * kObsChunk;
  const int o_end = o_begin + kObsChunk < o_last ? o_begin + kObsChunk : o_last;
  const bool live = e < A.n_edges;
  double px[NP], py[NP], pz[NP];
  double cx = 0.0, cy = 0.0, cz = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int64_t b = (int64_t)(live ? e : 0) * (3 * NP) + 3 * k;
    px[k] = A.P[b]; py[k] = A.P[b + 1]; pz[k] = A.P[b + 2];
    cx += px[k]; cy += py[k]; cz += pz[k];
  }
  cx /= NP; cy /= NP; cz /= NP;
  double scale = 1.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) scale = fmax(scale, fmax(fabs(px[k]), fmax(fabs(py[k]), fabs(pz[k]))));
  int collide = 0;
  for (int o = o_begin; o < o_end; ++o) {
    bool inside = false, beyond = false;
    if constexpr (!kPoly) {
      const double lx = A.box_lo[3 * o], ly = A.box_lo[3 * o + 1], lz = A.box_lo[3 * o + 2];
      const double hx = A.box_hi[3 * o], hy = A.box_hi[3 * o + 1], hz = A.box_hi[3 * o + 2];
      // step 1: a control point inside the (closed) box
#pragma unroll
      for (int k = 0; k < NP; ++k)
        inside |= (px[k] >= lx) & (px[k] <= hx) & (py[k] >= ly) & (py[k] <= hy) & (pz[k] >= lz) & (pz[k] <= hz);
      // step 2: supporting plane of the box with normal centroid - clamp(centroid)
      const double nx = cx - fmin(fmax(cx, lx), hx), ny = cy - fmin(fmax(cy, ly), hy), nz = cz - fmin(fmax(cz, lz), hz);
      const double l = (nx > 0.0 ? nx * hx : nx * lx) + (ny > 0.0 ? ny * hy : ny * ly) + (nz > 0.0 ? nz * hz : nz * lz);
      beyond = (nx != 0.0) | (ny != 0.0) | (nz != 0.0);
#pragma unroll
      for (int k = 0; k < NP; ++k) beyond &= (nx * px[k] + ny * py[k] + nz * pz[k]) > l;
    } else {
      const int j = o - A.n_box;
      // step 1: a control point that satisfies every row (bit k set: point k
      // violates some row)
      const int r0 = A.pob_off[j], r1 = A.pob_off[j + 1];
      unsigned outside = 0u;
      for (int r = r0; r < r1; ++r) {
        const double ax = A.pob_A[3 * r], ay = A.pob_A[3 * r + 1], az = A.pob_A[3 * r + 2], bb = A.pob_b[r];
#pragma unroll
        for (int k = 0; k < NP; ++k) outside |= ((ax * px[k] + ay * py[k] + az * pz[k]) > bb ? 1u : 0u) << k;
      }
      inside = outside != (1u << NP) - 1u;
      if (!inside) {
        // step 2: the point of O nearest the centroid c (GJK over the set
        // c - O, whose support is c minus the vertex maximising u . v); the
        // normal n = c - that point; offset = max over the vertices of n . v
        const int v0 = A.pv_off[j], v1 = A.pv_off[j + 1];
        const V3 c{cx, cy, cz};
        auto vmax = [&](V3 u, double& best) -> V3 {
          V3 bv{A.pv[3 * v0], A.pv[3 * v0 + 1], A.pv[3 * v0 + 2]};
          best = dot(u, bv);
          for (int q = v0 + 1; q < v1; ++q) {
            const V3 vq{A.pv[3 * q], A.pv[3 * q + 1], A.pv[3 * q + 2]};
            const double d = dot(u, vq);
            if (d > best) { best = d; bv = vq; }
          }
          return bv;
        };
        auto support = [&](V3 u) -> V3 { double bd; return sub(c, vmax(u, bd)); };
        V3 n;
        const V3 w0 = sub(c, V3{A.pv[3 * v0], A.pv[3 * v0 + 1], A.pv[3 * v0 + 2]});
        (void)gjk_dist2(support, w0, 1e-24 * scale * scale, n);
        double l;
        (void)vmax(n, l);
        beyond = (n.x != 0.0) | (n.y != 0.0) | (n.z != 0.0);
#pragma unroll
        for (int k = 0; k < NP; ++k) beyond &= (n.x * px[k] + n.y * py[k] + n.z * pz[k]) > l;
      }
    }
    int code, step;
    if (inside) { code = 0; step = 1; }
    else if (beyond) { code = 1; step = 2; }
    else { code = 0; step = 3; }
    const bool undecided = live && step == 3;
    // append the undecided pairs: one atomic per wavefront
    const unsigned long long mask = __ballot(undecided);
    if (mask) {
      const int lane = __lane_id();
      const int leader = __ffsll((long long)mask) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(A.counter, (unsigned long long)__popcll(mask));
      base = __shfl(base, leader, kWave);
      if (undecided) {
        const unsigned long long pos = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (pos < (unsigned long long)A.list_cap) A.list[pos] = ((int64_t)o << 32) | (int64_t)e;
      }
    }
    if (live) {
      const int64_t q = (int64_t)o * A.n_edges + e;
      A.code[q] = (uint8_t)code;
      if (A.step) A.step[q] = (uint8_t)step;
      if (A.qp_dist2) A.qp_dist2[q] = __builtin_nan("");
      collide += (step == 1) ? 1 : 0;
    }
  }
  if (live && collide) atomicAdd(&A.n_collide[e], collide);
}

// Closest point to the origin of the face of the simplex {w0..w3} selected
// by MASK (bits = vertices): the affine projection, accepted when its
// barycentric weights are all positive.  Every index is a compile-time
// constant, so the simplex stays in registers.
template <int MASK>
__device__ __forceinline__ bool face_point(const V3 (&w)[4], V3& x) {
  constexpr int S = __builtin_popcount(MASK);
  constexpr int I0 = (MASK & 1) ? 0 : (MASK & 2) ? 1 : (MASK & 4) ? 2 : 3;
  const V3 w0 = w[I0];
  if constexpr (S == 1) {
    x = w0;
    return true;
  } else {
    // the other vertices of the face, in increasing order
    V3 d[3];
    int m = 0;
#pragma unroll
    for (int i = I0 + 1; i < 4; ++i)
      if (MASK & (1 << i)) d[m++] = sub(w[i], w0);
    // minimise |w0 + sum_j t_j d_j|^2: Gram system G t = -D^T w0
    double G[3][3], rhs[3], t[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < S - 1; ++a) {
      rhs[a] = -dot(d[a], w0);
#pragma unroll
      for (int c = 0; c < S - 1; ++c) G[a][c] = dot(d[a], d[c]);
    }
    double scale = 0.0;
#pragma unroll
    for (int a = 0; a < S - 1; ++a) scale = fmax(scale, G[a][a]);
    if constexpr (S == 2) {
      if (!(G[0][0] > 1e-30 * fmax(scale, 1e-300))) return false;
      t[0] = rhs[0] / G[0][0];
    } else if constexpr (S == 3) {
      const double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
      if (!(fabs(det) > 1e-24 * scale * scale)) return false;
      t[0] = (rhs[0] * G[1][1] - G[0][1] * rhs[1]) / det;
      t[1] = (G[0][0] * rhs[1] - rhs[0] * G[1][0]) / det;
    } else {
      const double det = G[0][0] * (G[1][1] * G[2][2] - G[1][2] * G[2][1]) -
                         G[0][1] * (G[1][0] * G[2][2] - G[1][2] * G[2][0]) +
                         G[0][2] * (G[1][0] * G[2][1] - G[1][1] * G[2][0]);
      if (!(fabs(det) > 1e-24 * scale * scale * scale)) return false;
      // Cramer's rule, column c of G replaced by rhs
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double M[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int b = 0; b < 3; ++b) M[a][b] = (b == c) ? rhs[a] : G[a][b];
        t[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
      }
    }
    double t0 = 1.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < S - 1; ++j) {
      t0 -= t[j];
      ok &= t[j] > -1e-14;
    }
    if (!(ok && t0 > -1e-14)) return false;
    x = w0;
#pragma unroll
    for (int j = 0; j < S - 1; ++j) x = axpy(t[j], d[j], x);
    return true;
  }
}

template <int MASK>
__device__ __forceinline__ void try_face(const V3 (&w)[4], int k, double& best, int& best_mask, V3& best_v) {
  if (MASK >= (1 << k)) return;
  V3 x;
  if (!face_point<MASK>(w, x)) return;
  const double xx = dot(x, x);
  if (xx < best) { best = xx; best_mask = MASK; best_v = x; }
}

// keep the vertices of face MASK, in order, as the new simplex
template <int MASK>
__device__ __forceinline__ void keep_face(V3 (&w)[4], int& k) {
  V3 nw[4] = {w[0], w[0], w[0], w[0]};
  int s = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (MASK & (1 << i)) nw[s++] = w[i];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = nw[i];
  k = __builtin_popcount(MASK);
}

// Closest point to the origin of conv(w[0..k)), k <= 4: the nearest accepted
// face projection over every face.  On return w[0..k) holds that face.
// Returns false when no face qualified (degenerate input).
__device__ bool closest_face(V3 (&w)[4], int& k, V3& v) {
  double best = __builtin_huge_val();
  int bm = 0;
  V3 bv{0.0, 0.0, 0.0};
  try_face<1>(w, k, best, bm, bv);  try_face<2>(w, k, best, bm, bv);  try_face<3>(w, k, best, bm, bv);
  try_face<4>(w, k, best, bm, bv);  try_face<5>(w, k, best, bm, bv);  try_face<6>(w, k, best, bm, bv);
  try_face<7>(w, k, best, bm, bv);  try_face<8>(w, k, best, bm, bv);  try_face<9>(w, k, best, bm, bv);
  try_face<10>(w, k, best, bm, bv); try_face<11>(w, k, best, bm, bv); try_face<12>(w, k, best, bm, bv);
  try_face<13>(w, k, best, bm, bv); try_face<14>(w, k, best, bm, bv); try_face<15>(w, k, best, bm, bv);
  switch (bm) {
    case 1: keep_face<1>(w, k); break;   case 2: keep_face<2>(w, k); break;   case 3: keep_face<3>(w, k); break;
    case 4: keep_face<4>(w, k); break;   case 5: keep_face<5>(w, k); break;   case 6: keep_face<6>(w, k); break;
    case 7: keep_face<7>(w, k); break;   case 8: keep_face<8>(w, k); break;   case 9: keep_face<9>(w, k); break;
    case 10: keep_face<10>(w, k); break; case 11: keep_face<11>(w, k); break; case 12: keep_face<12>(w, k); break;
    case 13: keep_face<13>(w, k); break; case 14: keep_face<14>(w, k); break; case 15: keep_face<15>(w, k); break;
    default: return false;
  }
  v = bv;
  return true;
}

// Squared distance from the origin to a convex set given by its support
// mapping (support(u) minimises u . w over the set), starting from the point
// w0 of the set: the Gilbert-Johnson-Keerthi iteration, stopping when
// |v|^2 - v . w <= 1e-13 |v|^2 (the gap bound), when no progress is made or
// when the origin lies in a tetrahedron of set points.  Results at or below
// zero2 count as 0.  v returns the closest point found.
template <class Support>
__device__ double gjk_dist2(Support support, V3 w0, double zero2, V3& v) {
  V3 w[4] = {w0, w0, w0, w0};
  int k = 1;
  v = w0;
  double vv = dot(v, v);
  for (int it = 0; it < 64 && vv > zero2; ++it) {
    const V3 wn = support(v);
    if (vv - dot(v, wn) <= 1e-13 * vv) break;
    bool dup = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) dup |= (i < k) & (w[i].x == wn.x) & (w[i].y == wn.y) & (w[i].z == wn.z);
    if (dup) break;
    // append at slot k (fixed slots keep the simplex in registers)
    if (k == 1) w[1] = wn;
    else if (k == 2) w[2] = wn;
    else w[3] = wn;
    ++k;
    V3 nv;
    if (!closest_face(w, k, nv)) break;
    const double nvv = dot(nv, nv);
    if (!(nvv < vv)) break;   // no progress: v is optimal to rounding
    v = nv;
    vv = nvv;
    if (k == 4) { vv = 0.0; v = V3{0.0, 0.0, 0.0}; break; }   // the origin lies in a tetrahedron
  }
  return vv > zero2 ? vv : 0.0;
}

// ---- Cut-QP value of a polytope pair (one wavefront per pair)
//
// With the slacks eliminated (for fixed weights the best slack of a row is
// its violation) the Cut-QP optimum is  f* = min over x in conv(P) of
// f(x) = |(A x - b)_+|^2, a convex piecewise quadratic; on the rows S
// violated at x it equals q_S(x) = |A_S x - b_S|^2.  Each outer step
//   1. evaluates f and the Lagrange-dual bound h(mu) = min_j mu . (A P_j - b)
//      - |mu|^2 / 4 <= f* at mu = 2 (A x - b)_+, and stops when f - h is at
//      most 1e-11 f or f no longer decreases;
//   2. minimises q_S over conv(P) exactly (Wolfe's minimum-norm-point method:
//      q_S(P^T lam) is the squared norm of sum_j lam_j w_j with
//      w_j = A_S P_j - b_S, whose Gram matrix follows from the moments
//      H = A_S^T A_S, g = A_S^T b_S, c = |b_S|^2);
//   3. moves to the minimiser of f on the segment towards that point (f is a
//      convex piecewise quadratic along it: safeguarded Newton on its slope,
//      exact once the segment's violated rows are found).
// Once S is the violated set of the optimum, step 2 lands on it.  The rows
// are spread one per lane (at most 32); x and the moments are uniform.

// 3 x 3 symmetric matrix as (xx, xy, xz, yy, yz, zz)
__device__ __forceinline__ V3 sym_mul(const double (&H)[6], V3 v) {
  return {H[0] * v.x + H[1] * v.y + H[2] * v.z, H[1] * v.x + H[3] * v.y + H[4] * v.z,
          H[2] * v.x + H[4] * v.y + H[5] * v.z};
}

// Wolfe's minimum-norm-point method for min over the simplex of
// q(x) = x^T H x - 2 g^T x + c, x = sum_j lam_j P_j, H positive
// semidefinite.  q is the squared norm of sum_j lam_j w_j for points w_j of
// an affine space of dimension at most 3, so the corral (the affinely
// independent points carrying the current weights) holds at most four; its
// points, weights and indices stay in registers.  Returns the minimiser x.
template <int NP>
__device__ V3 min_norm_point(const V3 (&pts)[NP], const double (&H)[6], V3 g, double c) {
  V3 cp[4];
  int cid[4];
  double al[4];
  // start at the vertex with the smallest q
  double qbest = __builtin_huge_val(), dmax = 0.0;
  cp[0] = pts[0];
  cid[0] = 0;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double qk = dot(pts[k], sym_mul(H, pts[k])) - 2.0 * dot(g, pts[k]) + c;
    dmax = fmax(dmax, fabs(qk));
    if (qk < qbest) { qbest = qk; cp[0] = pts[k]; cid[0] = k; }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) al[i] = i == 0 ? 1.0 : 0.0;
#pragma unroll
  for (int i = 1; i < 4; ++i) { cp[i] = cp[0]; cid[i] = -1; }
  int nc = 1;
  auto point = [&]() {
    V3 x{0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < 4; ++i) x = axpy(i < nc ? al[i] : 0.0, cp[i], x);
    return x;
  };
  bool done = false;
  for (int major = 0; major < 16 && !done; ++major) {
    const V3 x = point();
    const V3 v = sub(sym_mul(H, x), g);   // x_w . w_j = v . P_j - g . x + c
    const double gx = dot(g, x);
    const double xx = dot(v, x) - gx + c;
    double best = __builtin_huge_val();
    int jb = -1;
    V3 pb = pts[0];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const double vk = dot(v, pts[k]);
      if (vk < best) { best = vk; jb = k; pb = pts[k]; }
    }
    if (best - gx + c >= xx - 1e-14 * dmax) break;     // x is optimal
    bool dup = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) dup |= (i < nc) & (cid[i] == jb);
    if (dup || nc == 4) break;                         // no independent point left (rounding)
#pragma unroll
    for (int i = 1; i < 4; ++i)
      if (i == nc) { cp[i] = pb; cid[i] = jb; al[i] = 0.0; }
    ++nc;
    // minor cycles: the affine minimiser of the corral, clipped back into
    // its hull while it has a weight <= 0
    for (int minor = 0; minor < 4; ++minor) {
      // y minimises q(cp0 + sum_i y_i (cp_i - cp0)): [D^T H D] y = -D^T (H cp0 - g)
      const int n = nc - 1;
      V3 D[3];
      double M[3][3], y[3];
      const V3 r0 = sub(sym_mul(H, cp[0]), g);
#pragma unroll
      for (int i = 0; i < 3; ++i) D[i] = sub(cp[i + 1], cp[0]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const V3 HDi = sym_mul(H, D[i]);
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i][j] = (i < n && j < n) ? dot(D[j], HDi) : (i == j ? 1.0 : 0.0);
        y[i] = i < n ? -dot(D[i], r0) : 0.0;
      }
      // symmetric elimination (no pivoting: M is positive definite when the
      // corral is affinely independent); a pivot that vanishes against its
      // diagonal entry means it is not
      double d0[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) d0[i] = M[i][i];
      bool sing = false;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sing |= !(M[k][k] > 1e-12 * d0[k]) | !(d0[k] > 0.0);
        const double piv = M[k][k] > 0.0 ? M[k][k] : 1.0;
#pragma unroll
        for (int i = k + 1; i < 3; ++i) {
          const double l = M[i][k] / piv;
#pragma unroll
          for (int j = k + 1; j < 3; ++j) M[i][j] -= l * M[k][j];
          y[i] -= l * y[k];
        }
      }
#pragma unroll
      for (int k = 2; k >= 0; --k) {
        double acc = y[k];
#pragma unroll
        for (int j = k + 1; j < 3; ++j) acc -= M[k][j] * y[j];
        y[k] = acc / (M[k][k] > 0.0 ? M[k][k] : 1.0);
      }
      if (sing) {                                       // drop the last point, stop
        --nc;
        done = true;
        break;
      }
      double be[4];
      be[0] = 1.0;
#pragma unroll
      for (int i = 1; i < 4; ++i) { be[i] = i < nc ? y[i - 1] : 0.0; be[0] -= be[i]; }
      bool inside = true;
#pragma unroll
      for (int i = 0; i < 4; ++i) inside &= (i >= nc) | (be[i] > 0.0);
      if (inside) {
#pragma unroll
        for (int i = 0; i < 4; ++i) al[i] = be[i];
        break;
      }
      // largest step from al towards be that keeps every weight >= 0
      double th = 1.0;
      int kd = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (i < nc && be[i] <= 0.0) {
          const double ti = al[i] / (al[i] - be[i]);
          if (ti < th) { th = ti; kd = i; }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) al[i] = (1.0 - th) * al[i] + th * be[i];
      // remove corral point kd (its weight is now 0)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (i >= kd) { cp[i] = cp[i + 1]; cid[i] = cid[i + 1]; al[i] = al[i + 1]; }
      --nc;
      double sa = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) { al[i] = i < nc ? fmax(al[i], 0.0) : 0.0; sa += al[i]; }
#pragma unroll
      for (int i = 0; i < 4; ++i) al[i] /= sa;
      if (nc == 1) break;
    }
  }
  return point();
}

template <int NP>
__global__ __launch_bounds__(kCutBlock) void cut_value_kernel(CutArgs A) {
  const unsigned long long cnt = *A.counter;
  const int64_t n = (int64_t)(cnt < (unsigned long long)A.list_cap ? cnt : (unsigned long long)A.list_cap);
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kCutBlock / kWave) + threadIdx.x / kWave));
  const int64_t nw = (int64_t)gridDim.x * (kCutBlock / kWave);
  for (int64_t t = wv; t < n; t += nw) {
    const int64_t ent = A.list[t];
    const int o = (int)(ent >> 32), e = (int)(ent & 0xffffffffll);
    if (o < A.n_box) continue;
    const int64_t qi = (int64_t)o * A.n_edges + e;
    if (!(A.qp_dist2[qi] > 0.0)) continue;   // conv(P) meets O: the optimum is 0
    const int jp = o - A.n_box;
    const int r0 = A.pob_off[jp], m = A.pob_off[jp + 1] - r0;
    // row of this lane (idle lanes: 0 . x - 1 < 0, never violated)
    const bool rl = lane < m;
    const V3 a = rl ? V3{A.pob_A[3 * (r0 + lane)], A.pob_A[3 * (r0 + lane) + 1], A.pob_A[3 * (r0 + lane) + 2]}
                    : V3{0.0, 0.0, 0.0};
    const double bk = rl ? A.pob_b[r0 + lane] : 1.0;
    V3 pts[NP];
    V3 x{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int64_t b = (int64_t)e * (3 * NP) + 3 * k;
      pts[k] = {A.P[b], A.P[b + 1], A.P[b + 2]};
      x = axpy(1.0 / NP, pts[k], x);
    }
    double fbest = __builtin_huge_val(), fprev = __builtin_huge_val();
    for (int it = 0; it < 32; ++it) {
      const double r = dot(a, x) - bk;
      const double rp = fmax(r, 0.0);
      double s4[4] = {rp * rp, rp * a.x, rp * a.y, rp * a.z};
      wave::sum4(s4);
      const double f = s4[0];
      const double beta = wave::sum(rp * bk);
      fbest = fmin(fbest, f);
      if (!(f > 0.0) || !(f < fprev)) break;
      fprev = f;
      const V3 u{s4[1], s4[2], s4[3]};
      double mn = __builtin_huge_val();
#pragma unroll
      for (int k = 0; k < NP; ++k) mn = fmin(mn, dot(u, pts[k]));
      const double h = 2.0 * (mn - beta) - f;
      if (f - h <= 1e-11 * f) break;
      // moments of the violated rows
      const double sw = r > 0.0 ? 1.0 : 0.0;
      double m1[4] = {sw * a.x * a.x, sw * a.x * a.y, sw * a.x * a.z, sw * a.y * a.y};
      double m2[4] = {sw * a.y * a.z, sw * a.z * a.z, sw * bk * a.x, sw * bk * a.y};
      double m3[4] = {sw * bk * a.z, sw * bk * bk, 0.0, 0.0};
      wave::sum4(m1);
      wave::sum4(m2);
      wave::sum4(m3);
      const double H[6] = {m1[0], m1[1], m1[2], m1[3], m2[0], m2[1]};
      const V3 xs = min_norm_point<NP>(pts, H, V3{m2[2], m2[3], m3[0]}, m3[1]);
      // half the slope of f at x along xs - x is u . (xs - x): stop unless it
      // descends
      if (!(dot(u, sub(xs, x)) < 0.0)) break;
      // line search on f along x + t (xs - x), t in [0, 1]: half its slope
      // is sum_k (r_k + t d_k)_+ d_k, nondecreasing in t
      const double dk = dot(a, sub(xs, x));
      auto slope = [&](double t, double& s2) {
        const double rt = r + t * dk;
        double v2[2] = {rt > 0.0 ? rt * dk : 0.0, rt > 0.0 ? dk * dk : 0.0};
        // two sums, interleaved through the same stages
        double v4[4] = {v2[0], v2[1], 0.0, 0.0};
        wave::sum4(v4);
        s2 = v4[1];
        return v4[0];
      };
      double s2;
      double t = 1.0;
      const double g1 = slope(1.0, s2);
      if (g1 > 0.0) {
        double lo = 0.0, hi = 1.0;
        // the piece at t = 1 is linear: its root is the Newton point
        double tn = s2 > 0.0 ? 1.0 - g1 / s2 : 0.5;
        for (int ls = 0; ls < 40; ++ls) {
          t = (tn > lo && tn < hi) ? tn : 0.5 * (lo + hi);
          double q2;
          const double gt = slope(t, q2);
          if (gt == 0.0) break;
          if (gt > 0.0) hi = t; else lo = t;
          if (!(hi - lo > 1e-15)) break;
          tn = q2 > 0.0 ? t - gt / q2 : 0.5 * (lo + hi);
          if (tn == t) break;
        }
      }
      if (!(t > 0.0)) break;
      x = axpy(t, sub(xs, x), x);
    }
    if (lane == 0) A.qp_dist2[qi] = fbest;
  }
}

// Step 3 for every listed pair: squared distance between conv(P) and the box.
template <int P>
__global__ __launch_bounds__(kCutBlock) void cut_qp_kernel(CutArgs A) {
  constexpr int NP = P + 1;
  const unsigned long long cnt = *A.counter;
  const int64_t n = (int64_t)(cnt < (unsigned long long)A.list_cap ? cnt : (unsigned long long)A.list_cap);
  for (int64_t t = (int64_t)blockIdx.x * kCutBlock + threadIdx.x; t < n; t += (int64_t)gridDim.x * kCutBlock) {
    const int64_t ent = A.list[t];
    const int o = (int)(ent >> 32), e = (int)(ent & 0xffffffffll);
    V3 pts[NP];
    double scale = 1.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const int64_t b = (int64_t)e * (3 * NP) + 3 * k;
      pts[k] = {A.P[b], A.P[b + 1], A.P[b + 2]};
      scale = fmax(scale, fmax(fabs(pts[k].x), fmax(fabs(pts[k].y), fabs(pts[k].z))));
    }
    const double zero2 = 1e-24 * scale * scale;
    double d2, value;
    if (o < A.n_box) {
      const V3 lo{A.box_lo[3 * o], A.box_lo[3 * o + 1], A.box_lo[3 * o + 2]};
      const V3 hi{A.box_hi[3 * o], A.box_hi[3 * o + 1], A.box_hi[3 * o + 2]};
      // support point of conv(P) - box minimising u . w (kept by selection)
      auto support = [&](V3 u) -> V3 {
        V3 bp = pts[0];
        double bd = dot(u, pts[0]);
#pragma unroll
        for (int k = 1; k < NP; ++k) {
          const double d = dot(u, pts[k]);
          if (d < bd) { bd = d; bp = pts[k]; }
        }
        const V3 bx{u.x > 0.0 ? hi.x : lo.x, u.y > 0.0 ? hi.y : lo.y, u.z > 0.0 ? hi.z : lo.z};
        return sub(bp, bx);
      };
      const V3 c0{fmin(fmax(pts[0].x, lo.x), hi.x), fmin(fmax(pts[0].y, lo.y), hi.y), fmin(fmax(pts[0].z, lo.z), hi.z)};
      V3 v;
      d2 = gjk_dist2(support, sub(pts[0], c0), zero2, v);
      value = d2;   // unit rows: the Cut-QP optimum is the squared distance
    } else {
      const int jp = o - A.n_box;
      const int v0 = A.pv_off[jp], v1 = A.pv_off[jp + 1];
      // support point of conv(P) - conv(vertices) minimising u . w
      auto support = [&](V3 u) -> V3 {
        V3 bp = pts[0];
        double bd = dot(u, pts[0]);
#pragma unroll
        for (int k = 1; k < NP; ++k) {
          const double d = dot(u, pts[k]);
          if (d < bd) { bd = d; bp = pts[k]; }
        }
        V3 bv{A.pv[3 * v0], A.pv[3 * v0 + 1], A.pv[3 * v0 + 2]};
        double best = dot(u, bv);
        for (int q2 = v0 + 1; q2 < v1; ++q2) {
          const V3 vq{A.pv[3 * q2], A.pv[3 * q2 + 1], A.pv[3 * q2 + 2]};
          const double d = dot(u, vq);
          if (d > best) { best = d; bv = vq; }
        }
        return sub(bp, bv);
      };
      V3 v;
      d2 = gjk_dist2(support, sub(pts[0], V3{A.pv[3 * v0], A.pv[3 * v0 + 1], A.pv[3 * v0 + 2]}), zero2, v);
      // 0 when conv(P) meets O; otherwise the value pass overwrites it with
      // the Cut-QP optimum
      value = d2;
    }
    const int64_t q = (int64_t)o * A.n_edges + e;
    const int code = d2 > 0.0 ? 1 : 0;
    A.code[q] = (uint8_t)code;
    if (A.qp_dist2) A.qp_dist2[q] = value;
    if (!code) atomicAdd(&A.n_collide[e], 1);
  }
}

template <int P>
hipError_t launch_cut_p(const CutArgs& a, hipStream_t s, int qp_blocks) {
  const int gx = (a.n_edges + kCutBlock - 1) / kCutBlock;
  const int n_poly = a.n_obst - a.n_box;
  if (a.n_box > 0)
    hipLaunchKernelGGL((cut_prefilter_kernel<P, false>), dim3(gx, (a.n_box + kObsChunk - 1) / kObsChunk),
                       dim3(kCutBlock), 0, s, a);
  if (n_poly > 0)
    hipLaunchKernelGGL((cut_prefilter_kernel<P, true>), dim3(gx, (n_poly + kObsChunk - 1) / kObsChunk),
                       dim3(kCutBlock), 0, s, a);
  hipLaunchKernelGGL((cut_qp_kernel<P>), dim3(qp_blocks), dim3(kCutBlock), 0, s, a);
  if (a.qp_dist2 && n_poly > 0)
    hipLaunchKernelGGL((cut_value_kernel<P + 1>), dim3(qp_blocks), dim3(kCutBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cut(const CutArgs& a, hipStream_t s, int qp_blocks) {
  if (a.n_edges <= 0) return hipSuccess;
  hipLaunchKernelGGL(cut_zero_kernel, dim3((a.n_edges + kCutBlock - 1) / kCutBlock), dim3(kCutBlock), 0, s,
                     a.counter, a.n_collide, a.n_edges);
  if (a.n_obst <= 0) return hipGetLastError();
  switch (a.degree) {
    case 1: return launch_cut_p<1>(a, s, qp_blocks);
    case 2: return launch_cut_p<2>(a, s, qp_blocks);
    case 3: return launch_cut_p<3>(a, s, qp_blocks);
    case 4: return launch_cut_p<4>(a, s, qp_blocks);
    case 5: return launch_cut_p<5>(a, s, qp_blocks);
    case 6: return launch_cut_p<6>(a, s, qp_blocks);
    case 7: return launch_cut_p<7>(a, s, qp_blocks);
    case 8: return launch_cut_p<8>(a, s, qp_blocks);
    case 9: return launch_cut_p<9>(a, s, qp_blocks);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rbp
