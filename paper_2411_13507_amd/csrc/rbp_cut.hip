// Cutting graph edges against box obstacles (Sec. III-B, Alg. 2, eq. Cut-QP).
//
// A pair is an edge (control points P_0..P_p of its Bezier curve) and an
// axis-aligned box obstacle lo <= x <= hi.  By the convex-hull property
// (Property 1) the curve is free of the box when conv(P) and the box are
// disjoint.  Alg. 2 decides this in three steps:
//   1. a control point inside the box            -> 0 (may collide);
//   2. the box's supporting plane with normal n = centroid - clamp(centroid)
//      has every control point strictly beyond it -> 1 (free);
//   3. otherwise the Cut-QP: |delta*|^2 > 0       -> 1, else 0.
// For a box the Cut-QP's optimal slack is delta = (A x - b)_+ at the best
// x in conv(P), whose squared norm is the squared Euclidean distance from x
// to the box, so |delta*|^2 = dist(conv(P), box)^2.  Step 3 computes that
// distance with the Gilbert-Johnson-Keerthi iteration on the Minkowski
// difference conv(P) - box (support points in closed form), in FP64.
//
// Work split: steps 1-2 run for every pair, one thread per (edge, chunk of
// obstacles), control points in registers and the box of the current
// obstacle read with uniform (scalar) loads; codes are written
// obstacle-major so a wavefront's stores are contiguous.  Pairs left
// undecided (a fraction of a percent on cluttered graphs) are appended to a
// list with one atomic per wavefront, and a grid-stride kernel runs step 3
// on the list.
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

// Steps 1 and 2 of Alg. 2 for the pairs (e, o), o in this thread's chunk.
template <int P>
__global__ __launch_bounds__(kCutBlock) void cut_prefilter_kernel(CutArgs A) {
  constexpr int NP = P + 1;
  const int e = blockIdx.x * kCutBlock + threadIdx.x;
  const int o_begin = blockIdx.y * kObsChunk;
  const int o_end = o_begin + kObsChunk < A.n_obst ? o_begin + kObsChunk : A.n_obst;
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
  int collide = 0;
  for (int o = o_begin; o < o_end; ++o) {
    const double lx = A.box_lo[3 * o], ly = A.box_lo[3 * o + 1], lz = A.box_lo[3 * o + 2];
    const double hx = A.box_hi[3 * o], hy = A.box_hi[3 * o + 1], hz = A.box_hi[3 * o + 2];
    // step 1: a control point inside the (closed) box
    bool inside = false;
#pragma unroll
    for (int k = 0; k < NP; ++k)
      inside |= (px[k] >= lx) & (px[k] <= hx) & (py[k] >= ly) & (py[k] <= hy) & (pz[k] >= lz) & (pz[k] <= hz);
    // step 2: supporting plane of the box with normal centroid - clamp(centroid)
    const double nx = cx - fmin(fmax(cx, lx), hx), ny = cy - fmin(fmax(cy, ly), hy), nz = cz - fmin(fmax(cz, lz), hz);
    const double l = (nx > 0.0 ? nx * hx : nx * lx) + (ny > 0.0 ? ny * hy : ny * ly) + (nz > 0.0 ? nz * hz : nz * lz);
    bool beyond = (nx != 0.0) | (ny != 0.0) | (nz != 0.0);
#pragma unroll
    for (int k = 0; k < NP; ++k) beyond &= (nx * px[k] + ny * py[k] + nz * pz[k]) > l;
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

// Closest point to the origin of conv(W[0..k)), k <= 4, by checking every
// face of the simplex: the affine projection onto a face whose barycentric
// weights are all positive is a candidate, and the nearest candidate is the
// answer.  On return W holds the vertices of that face (k updated).
// Returns false when no face qualified (degenerate input).
__device__ bool closest_face(V3* W, int& k, V3& v) {
  double best = __builtin_huge_val();
  int best_mask = 0;
  V3 best_v{0, 0, 0};
  const int full = (1 << k) - 1;
  for (int mask = 1; mask <= full; ++mask) {
    int idx[4], s = 0;
    for (int i = 0; i < k; ++i)
      if (mask & (1 << i)) idx[s++] = i;
    V3 x;
    bool ok = true;
    if (s == 1) {
      x = W[idx[0]];
    } else {
      // minimise |w0 + sum_j t_j d_j|^2: Gram system G t = -D^T w0
      const V3 w0 = W[idx[0]];
      V3 d[3];
      for (int j = 1; j < s; ++j) d[j - 1] = sub(W[idx[j]], w0);
      const int m = s - 1;
      double G[3][3], rhs[3], t[3] = {0, 0, 0};
      for (int a = 0; a < m; ++a) {
        rhs[a] = -dot(d[a], w0);
        for (int c = 0; c < m; ++c) G[a][c] = dot(d[a], d[c]);
      }
      double scale = 0.0;
      for (int a = 0; a < m; ++a) scale = fmax(scale, G[a][a]);
      if (m == 1) {
        if (!(G[0][0] > 1e-30 * fmax(scale, 1e-300))) ok = false;
        else t[0] = rhs[0] / G[0][0];
      } else if (m == 2) {
        const double det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
        if (!(fabs(det) > 1e-24 * scale * scale)) ok = false;
        else {
          t[0] = (rhs[0] * G[1][1] - G[0][1] * rhs[1]) / det;
          t[1] = (G[0][0] * rhs[1] - rhs[0] * G[1][0]) / det;
        }
      } else {
        const double c00 = G[1][1] * G[2][2] - G[1][2] * G[2][1];
        const double c01 = G[1][2] * G[2][0] - G[1][0] * G[2][2];
        const double c02 = G[1][0] * G[2][1] - G[1][1] * G[2][0];
        const double det = G[0][0] * c00 + G[0][1] * c01 + G[0][2] * c02;
        if (!(fabs(det) > 1e-24 * scale * scale * scale)) ok = false;
        else {
          // Cramer's rule
          for (int col = 0; col < 3; ++col) {
            double M[3][3];
            for (int a = 0; a < 3; ++a)
              for (int c = 0; c < 3; ++c) M[a][c] = (c == col) ? rhs[a] : G[a][c];
            const double dm = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                              M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                              M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
            t[col] = dm / det;
          }
        }
      }
      if (ok) {
        double t0 = 1.0;
        for (int j = 0; j < m; ++j) {
          t0 -= t[j];
          ok &= t[j] > -1e-14;
        }
        ok &= t0 > -1e-14;
        x = w0;
        for (int j = 0; j < m; ++j) x = axpy(t[j], d[j], x);
      }
    }
    if (!ok) continue;
    const double xx = dot(x, x);
    if (xx < best) { best = xx; best_mask = mask; best_v = x; }
  }
  if (best_mask == 0) return false;
  int s = 0;
  V3 keep[4];
  for (int i = 0; i < k; ++i)
    if (best_mask & (1 << i)) keep[s++] = W[i];
  for (int i = 0; i < s; ++i) W[i] = keep[i];
  k = s;
  v = best_v;
  return true;
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
    for (int k = 0; k < NP; ++k) {
      const int64_t b = (int64_t)e * (3 * NP) + 3 * k;
      pts[k] = {A.P[b], A.P[b + 1], A.P[b + 2]};
      scale = fmax(scale, fmax(fabs(pts[k].x), fmax(fabs(pts[k].y), fabs(pts[k].z))));
    }
    const V3 lo{A.box_lo[3 * o], A.box_lo[3 * o + 1], A.box_lo[3 * o + 2]};
    const V3 hi{A.box_hi[3 * o], A.box_hi[3 * o + 1], A.box_hi[3 * o + 2]};
    // support point of conv(P) - box minimising u . w
    auto support = [&](V3 u) -> V3 {
      int best = 0;
      double bv = dot(u, pts[0]);
      for (int k = 1; k < NP; ++k) {
        const double d = dot(u, pts[k]);
        if (d < bv) { bv = d; best = k; }
      }
      const V3 bx{u.x > 0.0 ? hi.x : lo.x, u.y > 0.0 ? hi.y : lo.y, u.z > 0.0 ? hi.z : lo.z};
      return sub(pts[best], bx);
    };
    V3 W[4];
    int k = 1;
    const V3 c0{fmin(fmax(pts[0].x, lo.x), hi.x), fmin(fmax(pts[0].y, lo.y), hi.y), fmin(fmax(pts[0].z, lo.z), hi.z)};
    W[0] = sub(pts[0], c0);
    V3 v = W[0];
    const double zero2 = 1e-24 * scale * scale;
    double vv = dot(v, v);
    for (int it = 0; it < 64 && vv > zero2; ++it) {
      const V3 w = support(v);
      // |v|^2 - v.w bounds the gap between |v|^2 and the squared distance
      if (vv - dot(v, w) <= 1e-13 * vv) break;
      bool dup = false;
      for (int i = 0; i < k; ++i) dup |= (W[i].x == w.x) & (W[i].y == w.y) & (W[i].z == w.z);
      if (dup) break;
      W[k++] = w;
      V3 nv;
      if (!closest_face(W, k, nv)) break;
      const double nvv = dot(nv, nv);
      if (!(nvv < vv)) break;   // no progress: v is optimal to rounding
      v = nv;
      vv = nvv;
      if (k == 4) { vv = 0.0; break; }   // the origin lies in a tetrahedron
    }
    const double d2 = vv > zero2 ? vv : 0.0;
    const int64_t q = (int64_t)o * A.n_edges + e;
    const int code = d2 > 0.0 ? 1 : 0;
    A.code[q] = (uint8_t)code;
    if (A.qp_dist2) A.qp_dist2[q] = d2;
    if (!code) atomicAdd(&A.n_collide[e], 1);
  }
}

template <int P>
hipError_t launch_cut_p(const CutArgs& a, hipStream_t s, int qp_blocks) {
  const dim3 g((a.n_edges + kCutBlock - 1) / kCutBlock, (a.n_obst + kObsChunk - 1) / kObsChunk);
  hipLaunchKernelGGL((cut_prefilter_kernel<P>), g, dim3(kCutBlock), 0, s, a);
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
