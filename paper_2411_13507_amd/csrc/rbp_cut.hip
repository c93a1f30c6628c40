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
// polytope the optimum itself is then computed by accelerated projected
// gradient on the convex weights, stopped by the Lagrange-dual gap.
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

// Euclidean projection of v onto the simplex {lam >= 0, sum lam = 1}: the
// threshold is max over k of (sum of the k largest entries - 1) / k, taken
// here over the sets {i : v_i >= v_j} (no sorting, constant indices).
template <int NP>
__device__ __forceinline__ void project_simplex(const double (&v)[NP], double (&out)[NP]) {
  double theta = -__builtin_huge_val();
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double sum = 0.0, cnt = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const bool in = v[i] >= v[j];
      sum += in ? v[i] : 0.0;
      cnt += in ? 1.0 : 0.0;
    }
    theta = fmax(theta, (sum - 1.0) / cnt);
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) out[i] = fmax(v[i] - theta, 0.0);
}

// Cut-QP optimum for the polytope rows r0..r1-1 of (Ar, br): the minimum over
// the convex weights lam of f = |(A P^T lam - b)_+|^2, by projected gradient
// with Nesterov momentum (step 1/L with L = 2 |A|_F^2 sum_k |P_k - mean|^2,
// a bound of the curvature along the simplex; momentum restarted when f
// rises), stopped when f is within 1e-10 f of the Lagrange-dual bound
// h(mu) = min_k mu . (A P_k - b) - |mu|^2 / 4 at mu = 2 (A x - b)_+, or after
// 4,000 steps.  Returns the smallest f seen (an upper bound of the optimum).
template <int NP>
__device__ double cut_qp_value(const V3 (&pts)[NP], const double* __restrict__ Ar, const double* __restrict__ br,
                               int r0, int r1) {
  V3 pm{0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < NP; ++k) pm = axpy(1.0 / NP, pts[k], pm);
  double sp = 0.0;
#pragma unroll
  for (int k = 0; k < NP; ++k) { const V3 d = sub(pts[k], pm); sp += dot(d, d); }
  double sa = 0.0;
  for (int r = r0; r < r1; ++r) sa += Ar[3 * r] * Ar[3 * r] + Ar[3 * r + 1] * Ar[3 * r + 1] + Ar[3 * r + 2] * Ar[3 * r + 2];
  // f, the row-weighted gradient A^T (A x - b)_+ and (A x - b)_+ . b at x
  auto eval = [&](V3 x, V3& gr, double& rb) -> double {
    double f = 0.0;
    gr = V3{0.0, 0.0, 0.0};
    rb = 0.0;
    for (int r = r0; r < r1; ++r) {
      const V3 a{Ar[3 * r], Ar[3 * r + 1], Ar[3 * r + 2]};
      const double s = fmax(dot(a, x) - br[r], 0.0);
      f += s * s;
      gr = axpy(s, a, gr);
      rb += s * br[r];
    }
    return f;
  };
  double lam[NP], y[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) { lam[k] = 1.0 / NP; y[k] = lam[k]; }
  auto point = [&](const double (&l)[NP]) -> V3 {
    V3 x{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < NP; ++k) x = axpy(l[k], pts[k], x);
    return x;
  };
  V3 gr;
  double rb;
  double fbest = eval(point(lam), gr, rb);
  if (!(sp > 0.0) || !(sa > 0.0) || fbest == 0.0) return fbest;
  const double inv_l = 1.0 / (2.0 * sa * sp);
  double t = 1.0, fprev = fbest;
  for (int it = 0; it < 4000; ++it) {
    (void)eval(point(y), gr, rb);
    double z[NP], ln[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) z[k] = y[k] - 2.0 * dot(gr, pts[k]) * inv_l;
    project_simplex<NP>(z, ln);
    const double f = eval(point(ln), gr, rb);
    double mn = __builtin_huge_val();
#pragma unroll
    for (int k = 0; k < NP; ++k) mn = fmin(mn, dot(gr, pts[k]));
    const double h = 2.0 * mn - 2.0 * rb - f;
    fbest = fmin(fbest, f);
    if (f - h <= 1e-10 * f) break;
    if (f > fprev) {                       // restart the momentum
      t = 1.0;
#pragma unroll
      for (int k = 0; k < NP; ++k) { y[k] = ln[k]; lam[k] = ln[k]; }
    } else {
      const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
      const double beta = (t - 1.0) / tn;
#pragma unroll
      for (int k = 0; k < NP; ++k) { y[k] = ln[k] + beta * (ln[k] - lam[k]); lam[k] = ln[k]; }
      t = tn;
    }
    fprev = f;
  }
  return fbest;
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
      // the value only when it is asked for (the decision needs d2 alone)
      value = (A.qp_dist2 && d2 > 0.0) ? cut_qp_value<NP>(pts, A.pob_A, A.pob_b, A.pob_off[jp], A.pob_off[jp + 1])
                                       : 0.0;
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
