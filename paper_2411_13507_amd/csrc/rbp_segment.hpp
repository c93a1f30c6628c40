// Device code of the batched segment QP for gfx950 (one 64-lane wavefront
// per instance), shared by the translation units that instantiate its
// kernels: rbp_kernels.hip (one wavefront per workgroup, one launch per
// degree group) and rbp_kernels_var.hip (the other launch shapes and the
// single-launch schedule).  Each unit holds its own copy of the per-degree
// constant table.
//
// Problem per instance (the per-edge curve of the paper's Bezier graph,
// Sec. III; reachable polytope of Theorem 2, convex-hull Property 1):
//   minimise   int_0^T |b''(t)|^2 dt  over the control points P_0..P_p
//   subject to A_f P_k <= b_f (all k), |p/T Delta P_k| <= vmax,
//              |p(p-1)/T^2 Delta^2 P_k| <= amax (componentwise),
//              H vec(P) <= h0 + G x0,  P_0 = x0[0:3],  P_p = goal.
//
// The kernel works in the frame shifted to P_0 on the interior points
// x = vec(P_1..P_{p-1}) - 1 (x) P_0 (n = 3(p-1) variables); the pinned points
// enter as constants.  Rows are evaluated on the full shifted vector
// y~ = [0, x, goal - P_0].
//
// Forward pass, per instance:
//   1. setup (FP64): row bounds, row scalings (1 / norm of the row in the
//      whitened metric x = L^-T v, P = L L^T), reachable-row Gram on MFMA;
//   2. ADMM (operator splitting, OSQP form with sigma = 0 since the reduced
//      Hessian is positive definite) in FP32 for a fixed number of
//      iterations; its (z, y) pair proposes an active set;
//   3. FP64 polish: the dual active-set method of Goldfarb and Idnani,
//      started from the ADMM proposal (made dual feasible first), ends at
//      the exact optimum or with a Farkas vector that is re-verified in FP64
//      against a box every feasible point must lie in;
//   4. FP64 KKT residuals, cost, write-back, stored active set for backward.
// The backward pass solves the adjoint KKT system on the stored active set.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "rbp_internal.hpp"
#include "rbp_wave.hpp"

namespace rbp {
namespace {

// per-degree constants (Bernstein Hessian, whitening factor, ...); each
// translation unit has its own copy, uploaded by its own upload function
__constant__ DegConst c_deg[kMaxDeg + 1];

constexpr int kWave = 64;
constexpr float kBigF = 1e30f;
constexpr int kSolved = 0, kInfeasible = 1, kMaxIter = 2, kPolishFailed = 3, kNumerical = 4,
              kInvalid = 5;

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Orders LDS accesses between the lanes of one wavefront.  kWS = false: a
// workgroup barrier (one wavefront per workgroup).  kWS = true: memory fences
// around a scheduling barrier but no s_barrier (a wavefront's LDS operations
// execute in program order), so that several wavefronts of one workgroup,
// each on its own instance, never wait for each other.
template <bool kWS>
__device__ __forceinline__ void bsync() {
  if constexpr (kWS) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  } else {
    __syncthreads();
  }
}

__device__ __forceinline__ double wsum(double v) { return wave::sum(v); }
__device__ __forceinline__ double wmax(double v) { return wave::max(v); }
__device__ __forceinline__ bool wany(bool b) { return __ballot(b) != 0ull; }
// arg-max / arg-min with the lowest id on ties; identical in every lane
__device__ __forceinline__ void wargmax(double& v, int& id) { wave::argmax(v, id); }
__device__ __forceinline__ void wargmin(double& v, int& id) { wave::argmin(v, id); }
__device__ __forceinline__ double sel3(int c, double a, double b, double d) {
  return c == 0 ? a : (c == 1 ? b : d);
}

template <typename Real>
struct Lds {
  double *Hd, *Af, *rowval, *ybuf, *qbuf, *vA, *vB, *vC, *vD, *vE, *scal, *acte, *actc, *lam;
  int *actid, *actside;
  Real *HfT, *Aff, *vbuf, *xb1, *xb2, *Kx;
  double *Q1, *Rm;
  double *cL1i, *cQ1, *cGd, *Rd;   // staged degree tables; reciprocal diagonal of R
  double *Ri;                      // R^-1 (upper triangular, same stride as R)
};

template <typename Real>
__device__ Lds<Real> carve(char* s, const LdsDims& D) {
  Lds<Real> L;
  L.Hd = (double*)(s + D.o_Hd);
  L.Af = (double*)(s + D.o_Af);
  L.rowval = (double*)(s + D.o_rowval);
  L.ybuf = (double*)(s + D.o_ybuf);
  L.qbuf = L.ybuf + D.ncol;
  L.vA = (double*)(s + D.o_vec);
  L.vB = L.vA + D.nmax;
  L.vC = L.vB + D.nmax;
  L.vD = L.vC + D.nmax;
  L.vE = L.vD + D.nmax;
  L.scal = (double*)(s + D.o_scal);
  L.acte = (double*)(s + D.o_acte);
  L.actc = L.acte + D.nmax;
  L.lam = (double*)(s + D.o_lam);
  L.actid = (int*)(s + D.o_actid);
  L.actside = (int*)(s + D.o_actside);
  L.HfT = (Real*)(s + D.o_Hf);
  L.Aff = (Real*)(s + D.o_Aff);
  L.vbuf = (Real*)(s + D.o_vbuf);
  L.xb1 = (Real*)(s + D.o_xb1);
  L.xb2 = (Real*)(s + D.o_xb2);
  L.Kx = (Real*)(s + D.o_Kx);
  L.Q1 = (double*)(s + D.o_Q1);
  L.Rm = (double*)(s + D.o_R);
  L.cL1i = (double*)(s + D.o_cst);
  L.cQ1 = L.cL1i + kMaxFree * kMaxFree;
  L.cGd = L.cQ1 + kMaxPts * kMaxPts;
  L.Rd = (double*)(s + D.o_Rd);
  L.Ri = (double*)(s + D.o_Ri);
  return L;
}

// Stride (elements) of the transposed reachable block H^T (free columns).
__device__ __forceinline__ int hft_stride(const LdsDims& D) { return D.r_cap | 1; }

// The value of x, opaque to the optimiser at this point: values derived from
// it (lane-dependent addresses and indices) are formed where they are used
// instead of being hoisted out of the polish loop and held in registers for
// its whole length (the loop runs at the 256-register limit).
__device__ __forceinline__ int opaque(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// whitening: (L^-1 a)_i for var i = 3s + c, a given on the free vars in ``a``;
// Li = rows of L1inv (stride kMaxFree, in LDS or constant memory; lower
// triangular with explicit zeros above the diagonal, so the full row can be
// summed: a is finite).  Fixed trip count, every load issued before the
// first product.
template <int P>
__device__ __forceinline__ double whiten_at(const double* Li, double T15, const double* a, int i_in) {
  constexpr int NFP = P - 1;
  const int i = opaque(i_in);
  const int s = i / 3, c = i - 3 * (i / 3);
  double w[NFP], x[NFP];
#pragma unroll
  for (int t = 0; t < NFP; ++t) { w[t] = Li[kMaxFree * s + t]; x[t] = a[3 * t + c]; }
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < NFP; ++t) acc += w[t] * x[t];
  return T15 * acc;
}
// un-whitening: (L^-T v)_i (column s of L1inv, zero above row s)
template <int P>
__device__ __forceinline__ double unwhiten_at(const double* Li, double T15, const double* v, int i_in) {
  constexpr int NFP = P - 1;
  const int i = opaque(i_in);
  const int s = i / 3, c = i - 3 * (i / 3);
  double w[NFP], x[NFP];
#pragma unroll
  for (int t = 0; t < NFP; ++t) { w[t] = Li[kMaxFree * t + s]; x[t] = v[3 * t + c]; }
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < NFP; ++t) acc += w[t] * x[t];
  return T15 * acc;
}

// --------------------------------------------------------------------------
// Instance description shared by the forward and backward passes.
// --------------------------------------------------------------------------
template <int P>
struct Inst {
  static constexpr int NFP = P - 1;       // interior control points
  static constexpr int N = 3 * NFP;       // free variables
  static constexpr int NC = 3 * (P + 1);  // coefficients of a full row
  static constexpr int ND = 6 * P - 3;    // difference rows (velocity, acceleration)
  // odd row strides (in doubles) of the LDS copies read one row per lane,
  // so that a lane-strided 64-bit access touches distinct banks
  static constexpr int NS = N | 1;        // basis Q1 and factor R
  static constexpr int HDS = NC | 1;      // reachable rows
  double T, T15, iT3, sv, sa, vmax, amax;
  double x0[6], P0[3], dg[3];
  int nf, r, F, RB, m, f0;
  int64_t r0, hb, po;

  // coefficient of row ``id`` on full-vector entry e = 3*pt + c (pt = 0..P)
  __device__ double coef(int id, int pt, int c, const double* Af, const double* Hd) const {
    if (id < F) {
      const int s = id / nf, j = id - s * nf;
      return (pt == s + 1) ? Af[3 * j + c] : 0.0;
    }
    if (id < F + 3 * P) {
      const int l = id - F, k = l / 3, cc = l - 3 * (l / 3);
      if (cc != c) return 0.0;
      return sv * (double(pt == k + 1) - double(pt == k));
    }
    if (id < RB) {
      const int l = id - F - 3 * P, k = l / 3, cc = l - 3 * (l / 3);
      if (cc != c) return 0.0;
      return sa * (double(pt == k + 2) - 2.0 * double(pt == k + 1) + double(pt == k));
    }
    return Hd[(id - RB) * HDS + 3 * pt + c];
  }

  // Entry i = 3t + c (t < P - 1) of the whitened normal L^-1 a of row ``id``
  // (uniform), a restricted to the free variables.  A face row has
  // coefficients on one interior point and a difference row on two or three
  // consecutive points of one coordinate, so theirs are combinations of
  // columns of L1inv (Li = row t of L1inv); a reachable row is whitened from
  // its LDS copy (Li0 = L1inv, row stride kMaxFree).
  __device__ double whitened(int id, int t, int c, int i, const double* Li0, const double* Af,
                             const double* Hd) const {
    constexpr int NFP = P - 1;
    const double* Li = Li0 + kMaxFree * t;
    if (id < F) {
      const int s = id / nf, j = id - s * nf;
      return T15 * Li[s] * Af[3 * j + c];
    }
    if (id < RB) {
      const int l = id - F;
      const bool vel = l < 3 * P;
      const int l2 = vel ? l : l - 3 * P, k = l2 / 3, cc = l2 - 3 * k;
      double u;
      if (vel) {   // sv (P_{k+1} - P_k): free points k and k - 1
        u = sv * ((k <= NFP - 1 ? Li[k < NFP ? k : 0] : 0.0) - (k >= 1 ? Li[k >= 1 ? k - 1 : 0] : 0.0));
      } else {     // sa (P_{k+2} - 2 P_{k+1} + P_k): free points k + 1, k, k - 1
        u = sa * ((k + 1 <= NFP - 1 ? Li[k + 1 < NFP ? k + 1 : 0] : 0.0) - 2.0 * Li[k] +
                  (k >= 1 ? Li[k >= 1 ? k - 1 : 0] : 0.0));
      }
      return c == cc ? T15 * u : 0.0;
    }
    return whiten_at<P>(Li0, T15, Hd + (id - RB) * HDS + 3, i);
  }
};

// Copy n doubles (rows of RL values) from global memory into LDS rows of
// stride LD, with eight loads in flight per lane before the first store (the
// instance's rows arrive in one or two HBM round trips instead of one per
// element).  Returns true if a value is not finite.
template <int RL, int LD>
__device__ __forceinline__ bool stage_rows(double* dst, const double* __restrict__ src, int n, int lane) {
  bool bad = false;
  for (int base = 0; base < n; base += 8 * kWave) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * kWave + lane;
      v[u] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + u * kWave + lane;
      if (e < n) {
        dst[e + (e / RL) * (LD - RL)] = v[u];
        bad |= !isfinite(v[u]);
      }
    }
  }
  return bad;
}

// Sum of x[i] * v[i], i < n: x a per-lane LDS row, v an LDS vector; every
// load is issued before the first product (the scheduler would otherwise
// keep only a few in flight at this register pressure).
template <int n>
__device__ __forceinline__ double dot_row(const double* x, const double* v) {
  double a[n], b[n];
#pragma unroll
  for (int i = 0; i < n; ++i) { a[i] = x[i]; b[i] = v[i]; }
  __builtin_amdgcn_sched_barrier(0);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < n; ++i) acc += a[i] * b[i];
  return acc;
}
// acc - sum over k < q of col[k * stride] * v[k] (q uniform), subtracted in
// order, loads issued six at a time (indices past q read entry q - 1 and are
// not used).
__device__ __forceinline__ double colsub_q(double acc, const double* col, int stride, const double* v, int q) {
  for (int k0 = 0; k0 < q; k0 += 6) {
    double a[6], b[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int k = k0 + u < q ? k0 + u : q - 1;
      a[u] = col[k * stride];
      b[u] = v[k];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if (k0 + u < q) acc -= a[u] * b[u];
  }
  return acc;
}
// Sum over lane <= k < q of row[k] * v[k] (the upper-triangular part of a
// row), in order, loads issued six at a time.
__device__ __forceinline__ double rowsum_upper_q(const double* row, const double* v, int lane, int q) {
  double acc = 0.0;
  for (int k0 = 0; k0 < q; k0 += 6) {
    double a[6], b[6];
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int k = k0 + u < q ? k0 + u : q - 1;
      a[u] = row[k];
      b[u] = v[k];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 6; ++u)
      if (k0 + u < q && k0 + u >= lane) acc += a[u] * b[u];
  }
  return acc;
}

// ==========================================================================
// Forward pass
// ==========================================================================
// kTag only gives each kernel that calls solve_instance its own
// instantiation: a device function with one caller is compiled into it,
// whereas one shared by several kernels may be called out of line, with its
// arguments in a private-memory frame.
template <int P, typename Real, bool kAdmm, bool kWS = false, int kTag = 0>
__device__ void solve_instance(const SolveArgs& A, const InstDesc& idesc, char* smem) {
  using I = Inst<P>;
  constexpr int NFP = I::NFP, N = I::N, NC = I::NC, ND = I::ND, NS = I::NS, HDS = I::HDS;
  const int lane = kWS ? int(threadIdx.x & (kWave - 1)) : int(threadIdx.x);
  const DegConst& K = c_deg[P];
  const LdsDims& D = A.dims;
  Lds<Real> L = carve<Real>(smem, D);
  const int HS = hft_stride(D);

  // every global load of the set-up depends only on the descriptor: they are
  // all issued before the first wait (staging barrier)
  const int inst = idesc.inst;
  I in;
  in.T = A.T[inst];
  in.f0 = idesc.f0;
  in.nf = idesc.nf;
  in.r0 = idesc.r0;
  in.r = idesc.r;
  in.hb = idesc.hb;
  in.po = idesc.po;
  in.F = NFP * in.nf;
  in.RB = in.F + ND;
  in.m = in.RB + in.r;
  in.vmax = A.vmax;
  in.amax = A.amax;
  bool bad = !(in.T > 0.0) || !(in.T < 1e300);
  for (int e = 0; e < 6; ++e) { in.x0[e] = A.x0[6 * (int64_t)inst + e]; bad |= !isfinite(in.x0[e]); }
  double gl[3];
  for (int e = 0; e < 3; ++e) { gl[e] = A.goal[3 * (int64_t)inst + e]; bad |= !isfinite(gl[e]); }
  for (int c = 0; c < 3; ++c) { in.P0[c] = in.x0[c]; in.dg[c] = gl[c] - in.x0[c]; }
  in.T15 = in.T * sqrt(in.T);
  in.iT3 = 1.0 / (in.T * in.T * in.T);
  in.sv = double(P) / in.T;
  in.sa = double(P) * (P - 1) / (in.T * in.T);
  const int nf = in.nf, r = in.r, F = in.F, RB = in.RB, m = in.m;

  auto finish_nan = [&](int status) {
    if (lane < NC) A.P_out[3 * in.po + lane] = __builtin_nan("");
    if (lane == 0) {
      A.cost_out[inst] = status == kInfeasible ? __builtin_huge_val() : __builtin_nan("");
      A.status_out[inst] = status;
      A.kkt_out[inst] = __builtin_nan("");
      if (A.iters_out) { A.iters_out[2 * inst] = 0; A.iters_out[2 * inst + 1] = 0; }
      if (A.store) { A.st_q[inst] = 0; A.fw_status[inst] = status; }
    }
  };

  // per-lane inputs of the row set-up, loaded ahead of the staging
  const double bj_in = lane < nf ? A.b_face[in.f0 + lane] : 0.0;
  double h0_in[2] = {0.0, 0.0}, g_in[2][6];
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int l = lane + kWave * sl;
    const bool on = l < r;
    h0_in[sl] = on ? A.h0[in.r0 + l] : 0.0;
#pragma unroll
    for (int e = 0; e < 6; ++e) g_in[sl][e] = on ? A.G[6 * (in.r0 + l) + e] : 0.0;
  }

  // debug option: poison the workgroup's LDS first, so that a read of a
  // value never written turns the outputs into NaN
  if (A.debug_fill) {
    double* w = reinterpret_cast<double*>(smem);
    for (int e = lane; e < D.bytes / 8; e += kWave) w[e] = __builtin_nan("");
    bsync<kWS>();
  }
  // ---- stage instance data in LDS
  bad |= stage_rows<NC, HDS>(L.Hd, A.H + in.hb, r * NC, lane);
  for (int e = lane; e < nf * 3; e += kWave) L.Af[e] = A.A_face[3 * (int64_t)in.f0 + e];
  if (lane < NC) {
    const int pt = lane / 3, c = lane - 3 * (lane / 3);
    L.ybuf[lane] = (pt == P) ? sel3(c, in.dg[0], in.dg[1], in.dg[2]) : 0.0;
  }
  // degree tables read with lane-dependent indices (the Hessian and the
  // difference-row Gram only for the ADMM matrix)
  for (int e = lane; e < kMaxFree * kMaxFree; e += kWave) L.cL1i[e] = (&K.L1inv[0][0])[e];
  for (int e = lane; e < kMaxPts * kMaxPts; e += kWave) L.cQ1[e] = (&K.Q1[0][0])[e];
  if constexpr (kAdmm) {
    for (int e = lane; e < kMaxFree * kMaxFree; e += kWave) L.cGd[e] = (&K.Gdiff[0][0])[e];
  }
  bsync<kWS>();

  // ---- face rows: lane j < nf owns face j on every interior point
  const bool fl = lane < nf;
  double fa0 = 0, fa1 = 0, fa2 = 0, fu = 0, fan = 1.0;
  bool fixed_viol = false;
  if (fl) {
    fa0 = L.Af[3 * lane]; fa1 = L.Af[3 * lane + 1]; fa2 = L.Af[3 * lane + 2];
    const double bj = bj_in;
    fu = bj - (fa0 * in.P0[0] + fa1 * in.P0[1] + fa2 * in.P0[2]);
    fan = sqrt(fa0 * fa0 + fa1 * fa1 + fa2 * fa2);
    bad |= !(fan > 0.0) || !isfinite(bj) || !isfinite(fan);
    // rows on the pinned points are constants
    const double gv = fa0 * in.dg[0] + fa1 * in.dg[1] + fa2 * in.dg[2];
    fixed_viol = (0.0 > fu) || (gv > fu);
  }
  // face-row scaling on point s: 1 / |L^-1 a| = ifan * rkappa[s]
  const double ifan = 1.0 / (in.T15 * fan);

  // ---- difference rows: lane l < ND
  const bool dl = lane < ND;
  const double sqT = sqrt(in.T), isT = 1.0 / sqT;
  int dk = 0, dc = 0;
  bool dvel = true;
  // a difference row holds its value in [dlo_of(), dbd]: [-dbd, dbd], or the
  // single value dbd on a pinned start-velocity lane (no extra register)
  const bool pinl = A.pin_v0 && lane < 3;
  auto dlo_of = [&](double bd) { return pinl ? bd : -bd; };
  double dsc = 0, dbd = 0, dcst = 0, ddn = 0;
  if (dl) {
    if (lane < 3 * P) {
      dk = lane / 3; dc = lane - 3 * dk; dvel = true; dsc = in.sv; dbd = in.vmax;
      dcst = (dk == P - 1) ? in.sv * sel3(dc, in.dg[0], in.dg[1], in.dg[2]) : 0.0;
      ddn = K.rwn_vel[dk] * isT;
      if (pinl) {
        // pinned start velocity: the first derivative point equals x0[3+c];
        // its speed bound is then a constant test
        dbd = sel3(dc, in.x0[3], in.x0[4], in.x0[5]);   // no dynamic index into a register array
        fixed_viol |= fabs(dbd) > in.vmax;
      }
    } else {
      const int l2 = lane - 3 * P;
      dk = l2 / 3; dc = l2 - 3 * dk; dvel = false; dsc = in.sa; dbd = in.amax;
      dcst = (dk == P - 2) ? in.sa * sel3(dc, in.dg[0], in.dg[1], in.dg[2]) : 0.0;
      ddn = sqT * K.rwn_acc[dk];
    }
  }
  // the velocity rows chained from both pinned ends bound every coordinate of
  // P_p - P_0 by vmax T: beyond that the instance is infeasible
  if (lane < 3) fixed_viol |= fabs(sel3(lane, in.dg[0], in.dg[1], in.dg[2])) > in.vmax * in.T * (1.0 + 1e-12);
  // ---- reachable rows: lane l owns rows l and l + 64
  double ru[2] = {0, 0}, rcst[2] = {0, 0}, rdn[2] = {0, 0};
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int l = lane + kWave * sl;
    if (l < r) {
      const double* hr = L.Hd + l * HDS;
      double b = h0_in[sl];
      for (int e = 0; e < 6; ++e) b += g_in[sl][e] * in.x0[e];
      double s0 = 0, s1 = 0, s2 = 0;
      for (int k = 0; k <= P; ++k) { s0 += hr[3 * k]; s1 += hr[3 * k + 1]; s2 += hr[3 * k + 2]; }
      b -= s0 * in.P0[0] + s1 * in.P0[1] + s2 * in.P0[2];
      ru[sl] = b;
      bad |= !isfinite(b);
      rcst[sl] = hr[3 * P] * in.dg[0] + hr[3 * P + 1] * in.dg[1] + hr[3 * P + 2] * in.dg[2];
      double nn = 0.0;
      for (int c = 0; c < 3; ++c)
        for (int t = 0; t < NFP; ++t) {
          double w = 0.0;
          for (int t2 = 0; t2 <= t; ++t2) w += K.L1inv[t][t2] * hr[3 * (t2 + 1) + c];
          nn += w * w;
        }
      const double wn = in.T15 * sqrt(nn);
      rdn[sl] = wn > 1e-300 ? 1.0 / wn : 0.0;
      L.rowval[RB + l] = rdn[sl];   // scratch use: row scalings for the Gram below
    }
  }
  if (wany(bad)) { finish_nan(kInvalid); return; }
  if (wany(fixed_viol)) { finish_nan(kInfeasible); return; }

  // ======================================================================
  // ADMM in precision Real
  // ======================================================================
  const int K_admm = kAdmm ? A.admm_iters : 0;
  const bool vl = lane < N;
  const int vs = lane / 3, vc = lane - 3 * (lane / 3);
  // rows proposed by the ADMM (z, y) for the polish's warm start: score |y|
  // per owned row, -1 when not proposed (packed key = 2*id + (side > 0))
  float sc_f[NFP], sc_d = -1.0f, sc_r[2] = {-1.0f, -1.0f};
  int side_d = 0;
#pragma unroll
  for (int s = 0; s < NFP; ++s) sc_f[s] = -1.0f;
  // the polish-only variant is compiled without the ADMM (its registers would
  // otherwise bound the occupancy of the whole kernel)
  if constexpr (kAdmm) {
    const Real rho = Real(A.rho), alpha = Real(A.alpha), irho = Real(1) / Real(A.rho);
    // var lane i < N: row i of M = K^{-1} (K = P + rho A^T D^2 A on the free
    // variables), linear term q_i
    Real Mrow[N];
    double qd = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) Mrow[j] = 0;
    if (K_admm > 0) {
      // face Gram (3x3 symmetric) of unit face normals
      double g00, g01, g02, g11, g12, g22;
      {
        const double w = fl ? 1.0 / (fan * fan) : 0.0;
        g00 = wsum(w * fa0 * fa0); g01 = wsum(w * fa0 * fa1); g02 = wsum(w * fa0 * fa2);
        g11 = wsum(w * fa1 * fa1); g12 = wsum(w * fa1 * fa2); g22 = wsum(w * fa2 * fa2);
      }
      // stage FP-Real copies of the rows used by the iteration
      for (int e = lane; e < r * N; e += kWave) {
        const int l = e / N, i = e - N * (e / N);
        L.HfT[i * HS + l] = Real(L.Hd[l * HDS + 3 + i]);
      }
      if (fl) { L.Aff[4 * lane] = Real(fa0); L.Aff[4 * lane + 1] = Real(fa1); L.Aff[4 * lane + 2] = Real(fa2); }
      {
        // Gram sum_l d_l^2 h_l h_l^T over reachable rows with v_mfma_f32_32x32x2f32:
        // A = B^T = scaled rows, two rows per instruction (lanes 0-31: row 2t,
        // lanes 32-63: row 2t+1; column = lane % 32).
        floatx16 acc;
#pragma unroll
        for (int g = 0; g < 16; ++g) acc[g] = 0.0f;
        const int col = lane & 31, half = lane >> 5;
        for (int t = 0; 2 * t < r; ++t) {
          const int l = 2 * t + half;
          float av = 0.0f;
          if (l < r && col < N) av = float(L.rowval[RB + l] * L.Hd[l * HDS + 3 + col]);
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, av, acc, 0, 0, 0);
        }
#pragma unroll
        for (int g = 0; g < 16; ++g) {
          const int i = 8 * (g >> 2) + 4 * half + (g & 3);
          if (i < N && col < N) L.Kx[i * N + col] = Real(A.rho * acc[g]);
        }
      }
      bsync<kWS>();
      // lane j < N assembles column j of K: Hessian and difference rows in
      // closed form, face blocks from the face Gram, reachable rows from above
      Real kc[N];
      {
        const double gfa = sel3(vc, g00, g01, g02), gfb = sel3(vc, g01, g11, g12), gfc = sel3(vc, g02, g12, g22);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const int si = i / 3, ci = i - 3 * (i / 3);
          kc[i] = 0;
          if (vl) {
            double v = 0.0;
            if (ci == vc)
              v = in.iT3 * (2.0 * L.cQ1[kMaxPts * (si + 1) + vs + 1] + double(A.rho) * L.cGd[kMaxFree * si + vs]);
            if (si == vs) v += double(A.rho) * in.iT3 / K.kappa[si] * (ci == 0 ? gfa : (ci == 1 ? gfb : gfc));
            kc[i] = Real(v) + L.Kx[i * N + lane];
          }
        }
      }
      // Gauss-Jordan sweep on the register columns (K is symmetric positive
      // definite: no pivoting); afterwards kc = column ``lane`` of -K^{-1}
#pragma unroll
      for (int k = 0; k < N; ++k) {
        Real pk[N];
#pragma unroll
        for (int i = 0; i < N; ++i) pk[i] = wave::bcast(kc[i], k);
        const Real invd = Real(1) / pk[k];
        const Real f = kc[k] * invd;
        const bool isk = lane == k;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          if (i == k) kc[i] = isk ? -invd : f;
          else kc[i] = isk ? pk[i] * invd : kc[i] - pk[i] * f;
        }
      }
      if (vl) {
#pragma unroll
        for (int j = 0; j < N; ++j) Mrow[j] = -kc[j];
        qd = 2.0 * in.iT3 * L.cQ1[kMaxPts * (vs + 1) + P] * sel3(vc, in.dg[0], in.dg[1], in.dg[2]);
      }
    }
    const Real qr = Real(qd);
    // scaled row data in Real
    Real ff[NFP], fhi[NFP], zf[NFP], yf[NFP];
    const Real fa0r = Real(fa0), fa1r = Real(fa1), fa2r = Real(fa2);
#pragma unroll
    for (int s = 0; s < NFP; ++s) {
      const double fdn = ifan * K.rkappa[s];
      ff[s] = Real(fdn); fhi[s] = fl ? Real(fdn * fu) : Real(kBigF);
      zf[s] = 0; yf[s] = 0;
    }
    const Real dd = Real(ddn);
    const Real dlo = dl ? Real(ddn * (dlo_of(dbd) - dcst)) : Real(-kBigF);
    const Real dhi = dl ? Real(ddn * (dbd - dcst)) : Real(kBigF);
    Real zd = 0, yd = 0;
    // stencil on the free vars (index -1: pinned point)
    int di0 = -1, di1 = -1, di2 = -1;
    Real dw0 = 0, dw1 = 0, dw2 = 0;
    if (dl) {
      if (dvel) {
        if (dk + 1 <= NFP) { di0 = 3 * dk + dc; dw0 = Real(dsc); }          // P_{k+1}
        if (dk >= 1) { di1 = 3 * (dk - 1) + dc; dw1 = Real(-dsc); }          // P_k
      } else {
        if (dk + 2 <= NFP) { di0 = 3 * (dk + 1) + dc; dw0 = Real(dsc); }    // P_{k+2}
        if (dk + 1 >= 1 && dk + 1 <= NFP) { di1 = 3 * dk + dc; dw1 = Real(-2.0 * dsc); }
        if (dk >= 1) { di2 = 3 * (dk - 1) + dc; dw2 = Real(dsc); }           // P_k
      }
    }
    Real rr[2], rhi[2], zr[2], yr[2];
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int l = lane + kWave * sl;
      rr[sl] = Real(rdn[sl]);
      rhi[sl] = (l < r) ? Real(rdn[sl] * (ru[sl] - rcst[sl])) : Real(kBigF);
      zr[sl] = 0; yr[sl] = 0;
    }
    auto upd = [&](Real& z, Real& y, Real zh, Real lo, Real hi) {
      const Real zrl = alpha * zh + (Real(1) - alpha) * z;
      Real zn = zrl + y * irho;
      zn = zn < lo ? lo : (zn > hi ? hi : zn);
      y += rho * (zrl - zn);
      z = zn;
    };
    for (int it = 0; it < K_admm; ++it) {
      // v = D (rho z - y), in row order
      if (fl) {
#pragma unroll
        for (int s = 0; s < NFP; ++s) L.vbuf[s * nf + lane] = ff[s] * (rho * zf[s] - yf[s]);
      }
      if (dl) L.vbuf[F + lane] = dd * (rho * zd - yd);
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const int l = lane + kWave * sl;
        if (l < r) L.vbuf[RB + l] = rr[sl] * (rho * zr[sl] - yr[sl]);
      }
      bsync<kWS>();
      if (vl) {
        // A^T v with four partial sums so that the LDS loads overlap
        Real t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        const int k = vs + 1;
        const Real* vf = L.vbuf + vs * nf;
        int j = 0;
        for (; j + 4 <= nf; j += 4) {
          t0 += L.Aff[4 * j + vc] * vf[j];
          t1 += L.Aff[4 * j + 4 + vc] * vf[j + 1];
          t2 += L.Aff[4 * j + 8 + vc] * vf[j + 2];
          t3 += L.Aff[4 * j + 12 + vc] * vf[j + 3];
        }
        for (; j < nf; ++j) t0 += L.Aff[4 * j + vc] * vf[j];
        const Real* hrow = L.HfT + lane * HS;
        const Real* vr = L.vbuf + RB;
        int l = 0;
#pragma unroll 2
        for (; l + 4 <= r; l += 4) {
          t0 += hrow[l] * vr[l];
          t1 += hrow[l + 1] * vr[l + 1];
          t2 += hrow[l + 2] * vr[l + 2];
          t3 += hrow[l + 3] * vr[l + 3];
        }
        for (; l < r; ++l) t0 += hrow[l] * vr[l];
        Real t = (t0 + t1) + (t2 + t3);
        t += Real(in.sv) * (L.vbuf[F + 3 * (k - 1) + vc] - L.vbuf[F + 3 * k + vc]);
        const int AB = F + 3 * P;
        if (k >= 2) t += Real(in.sa) * L.vbuf[AB + 3 * (k - 2) + vc];
        t -= Real(2.0 * in.sa) * L.vbuf[AB + 3 * (k - 1) + vc];
        if (k <= P - 2) t += Real(in.sa) * L.vbuf[AB + 3 * k + vc];
        L.xb1[lane] = t - qr;
      }
      bsync<kWS>();
      if (vl) {
        Real x = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) x += Mrow[j] * L.xb1[j];
        L.xb2[lane] = x;
      }
      bsync<kWS>();
      if (fl) {
#pragma unroll
        for (int s = 0; s < NFP; ++s) {
          const Real zh = ff[s] * (fa0r * L.xb2[3 * s] + fa1r * L.xb2[3 * s + 1] + fa2r * L.xb2[3 * s + 2]);
          upd(zf[s], yf[s], zh, Real(-kBigF), fhi[s]);
        }
      }
      if (dl) {
        Real v = 0;
        if (di0 >= 0) v += dw0 * L.xb2[di0];
        if (di1 >= 0) v += dw1 * L.xb2[di1];
        if (di2 >= 0) v += dw2 * L.xb2[di2];
        upd(zd, yd, dd * v, dlo, dhi);
      }
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const int l = lane + kWave * sl;
        if (l < r) {
          Real v = 0;
          for (int i = 0; i < N; ++i) v += L.HfT[i * HS + l] * L.xb2[i];
          upd(zr[sl], yr[sl], rr[sl] * v, Real(-kBigF), rhi[sl]);
        }
      }
    }
    // proposed active set from (z, y)
#pragma unroll
    for (int s = 0; s < NFP; ++s)
      sc_f[s] = (fl && (fhi[s] - zf[s] < yf[s])) ? float(fabs(double(yf[s]))) : -1.0f;
    if (dl) {
      if (dhi - zd < yd) { sc_d = float(fabs(double(yd))); side_d = 1; }
      else if (zd - dlo < -yd) { sc_d = float(fabs(double(yd))); side_d = -1; }
    }
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int l = lane + kWave * sl;
      sc_r[sl] = (l < r && (rhi[sl] - zr[sl] < yr[sl])) ? float(fabs(double(yr[sl]))) : -1.0f;
    }
  }
  bsync<kWS>();   // ADMM scratch is reused by the polish from here on

  // ======================================================================
  // FP64 polish: dual active set (Goldfarb-Idnani) in whitened coordinates
  // ======================================================================
  // row values on ybuf for every owned row; returns normalised violation
  // score of the most violated inactive row as (score, key).
  unsigned act_bits = 0u;   // bit s: face slot s; bit NFP: diff; bits NFP+1, NFP+2: reach slots
  int q = 0;
  double vw = 0.0;          // whitened point, lane i < N
  double lamr = 0.0;        // multiplier of active constraint ``lane`` (lane < q)
  int steps = 0;
  int status = kPolishFailed;
  const double ftol = A.feas_tol;

  // unconstrained minimiser in whitened coordinates: v0 = -L^-1 q
  double v0 = 0.0;
  if (vl) {
    double acc = 0.0;
#pragma unroll
    for (int t = 0; t < NFP; ++t) {
      const double w = L.cL1i[kMaxFree * vs + t] * K.Q1[t + 1][P];
      acc += (t <= vs) ? w : 0.0;
    }
    v0 = -in.T15 * 2.0 * in.iT3 * sel3(vc, in.dg[0], in.dg[1], in.dg[2]) * acc;
  }
  // Box that holds every feasible x: the velocity rows chained from both
  // pinned ends.  bc, bw: offset of its centre from the unconstrained
  // minimiser x_u = L^-T v0 (the straight line at constant speed: point k at
  // (k / p) dg) and its half-widths.
  double bc = 0.0, bw = 0.0;
  if (vl) {
    const int k = vs + 1;
    const double vv = in.vmax * in.T / P, dgc = sel3(vc, in.dg[0], in.dg[1], in.dg[2]);
    const double lo = fmax(-k * vv, dgc - (P - k) * vv), hi = fmin(k * vv, dgc + (P - k) * vv);
    bc = 0.5 * (lo + hi) - (double(k) / P) * dgc;
    bw = fmax(0.5 * (hi - lo), 0.0);
  }
  // Upper bound of the whitened objective 1/2 |L^T x - v0|^2 over the
  // feasible points; a dual value above it proves that none exists (weak
  // duality).  The objective equals the cost int |b''|^2 (its minimum over
  // the free points is 0: the straight line at constant speed), and two
  // bounds hold:
  //  * the acceleration rows bound every coordinate of every control point of
  //    b'' by amax, so |b''(t)|^2 <= 3 amax^2 (convex hull) and the cost is at
  //    most 3 amax^2 T;
  //  * over the box, with centre x_c, half-widths w and the unconstrained
  //    minimiser x_u = L^-T v0: |L^T x - v0| <= |L^T (x_c - x_u)| +
  //    |L^T (x - x_c)| and |L^T d|^2 = d^T P d <= sum_ij |P_ij| |d_i| |d_j|
  //    (P = 2 Q_ff).
  // The smaller is returned.
  auto box_bound = [&]() -> double {
    if (vl) { L.vD[lane] = bc; L.vE[lane] = bw; }
    bsync<kWS>();
    double pc = 0.0, pw = 0.0;
    if (vl) {
#pragma unroll
      for (int t = 0; t < NFP; ++t) {
        const double qv = L.cQ1[kMaxPts * (vs + 1) + t + 1];
        pc += qv * L.vD[3 * t + vc];
        pw += fabs(qv) * L.vE[3 * t + vc];
      }
    }
    const double cc = 2.0 * in.iT3 * wsum(bc * pc), ww = 2.0 * in.iT3 * wsum(bw * pw);
    const double rt = sqrt(fmax(cc, 0.0)) + sqrt(fmax(ww, 0.0));
    bsync<kWS>();
    return fmin(0.5 * rt * rt, 3.0 * in.amax * in.amax * in.T * (1.0 + 1e-12));
  };
  double Uw = box_bound();

  // --- owner helpers: key = 2*id + (side>0)
  auto slot_of = [&](int id_in, int& own_lane, int& bit) {   // id uniform
    const int id = __builtin_amdgcn_readfirstlane(id_in);
    if (id < F) { const int s = id / nf; own_lane = id - s * nf; bit = s; }
    else if (id < RB) { own_lane = id - F; bit = NFP; }
    else { const int l = id - RB; own_lane = l & 63; bit = NFP + 1 + (l >> 6); }
  };

  // whitened normal of constraint (id, side): lane i < N gets entry i (also
  // to vA), lanes i >= N get 0.  ``id`` is uniform.
  auto build_normal = [&](int id_in, int side) -> double {
    const int id = __builtin_amdgcn_readfirstlane(id_in);
    double a = 0.0;
    if (vl) {
      a = double(side) * in.whitened(id, vs, vc, lane, L.cL1i, L.Af, L.Hd);
      L.vA[lane] = a;
    }
    bsync<kWS>();
    return a;
  };

  // c = Q1 a, z = a - Q1^T c by classical Gram-Schmidt (a: vA in LDS and
  // a_own, the lane's entry), then r = R^-1 c; lane i < N keeps z_i, lane
  // k < q keeps c_k and r_k (c also in vC).  One pass leaves z orthogonal to
  // the basis up to about eps |a| / |z|; a second pass re-orthogonalises when
  // |z|^2 < 1e-2 |a|^2, i.e. when that loss could exceed about 10 eps (the
  // "twice is enough" threshold of 1/2 would take it on nearly half of the
  // steps here: face rows on neighbouring points are close in the whitened
  // metric).
  auto project = [&](double a_own, double& zz, double& aa, double& z_own, double& r_own, double& c_own) {
    c_own = lane < q ? dot_row<N>(L.Q1 + lane * NS, L.vA) : 0.0;
    if (lane < q) L.vC[lane] = c_own;
    bsync<kWS>();
    z_own = vl ? colsub_q(a_own, L.Q1 + lane, NS, L.vC, q) : 0.0;
    aa = wsum(a_own * a_own);
    zz = wsum(z_own * z_own);
    if (zz < 1e-2 * aa && q > 0) {
      if (vl) L.vB[lane] = z_own;
      bsync<kWS>();
      const double e_own = lane < q ? dot_row<N>(L.Q1 + lane * NS, L.vB) : 0.0;
      if (lane < q) L.vE[lane] = e_own;
      bsync<kWS>();
      z_own = vl ? colsub_q(z_own, L.Q1 + lane, NS, L.vE, q) : 0.0;
      c_own += e_own;
      if (lane < q) L.vC[lane] = c_own;
      zz = wsum(z_own * z_own);
      bsync<kWS>();
    }
    r_own = lane < q ? rowsum_upper_q(L.Ri + lane * NS, L.vC, lane, q) : 0.0;
  };

  // R^-1 rebuilt by back substitution after a downdate: lane j builds column
  // j (entries i <= j); each lane reads back only its own column
  auto ri_rebuild = [&]() {
    for (int i = q - 1; i >= 0; --i) {
      double acc = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double rik = L.Rm[i * NS + k], xk = L.Ri[k * NS + lane];
        acc -= (k > i && k <= lane && k < q) ? rik * xk : 0.0;
      }
      if (lane < q && i <= lane) L.Ri[i * NS + lane] = acc * L.Rd[i];
    }
    bsync<kWS>();
  };

  // append the projected direction as a new basis column (R gets c and |z|;
  // R^-1 gets -R^-1 c / |z| and 1/|z|, with rv = R^-1 c and c_own = c on
  // lanes < q, z_own = z on lanes < N)
  auto append = [&](double nz, int id, int side, double e_full, double c_full, double rv, double z_own,
                    double c_own) {
    const double inz = 1.0 / nz;
    if (vl) L.Q1[q * NS + lane] = z_own * inz;
    if (lane < q) {
      L.Rm[lane * NS + q] = c_own;
      L.Ri[lane * NS + q] = -rv * inz;
    }
    if (lane == 0) {
      L.Rm[q * NS + q] = nz;
      L.Rd[q] = inz;
      L.Ri[q * NS + q] = inz;
      L.actid[q] = id; L.actside[q] = side; L.acte[q] = e_full; L.actc[q] = c_full;
    }
    int ol, bit;
    slot_of(id, ol, bit);
    if (lane == ol) act_bits |= (1u << bit);
    ++q;
    bsync<kWS>();
  };

  // remove basis column kd: shift R columns, restore triangular form with
  // Givens rotations applied to R rows and Q1 columns, shift active data
  auto drop = [&](int kd) {
    constexpr int EPL = (N * N + kWave - 1) / kWave;
    const int ln = opaque(lane);
    {
      int own, bit;
      slot_of(L.actid[kd], own, bit);
      if (lane == own) act_bits &= ~(1u << bit);
    }
    double tmp[EPL];
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      const int e = ln + kWave * u;
      const int row = e / N, col = e - N * (e / N);
      tmp[u] = (e < N * N && row < q && col >= kd && col < q - 1) ? L.Rm[row * NS + col + 1] : 0.0;
    }
    int id_n = 0, sd_n = 0;
    double e_n = 0, c_n = 0;
    if (lane >= kd && lane < q - 1) {
      id_n = L.actid[lane + 1]; sd_n = L.actside[lane + 1]; e_n = L.acte[lane + 1]; c_n = L.actc[lane + 1];
    }
    const double lam_n = __shfl(lamr, (lane + 1) & 63, kWave);
    bsync<kWS>();
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      const int e = ln + kWave * u;
      const int row = e / N, col = e - N * (e / N);
      if (e < N * N && row < q && col >= kd && col < q - 1) L.Rm[row * NS + col] = tmp[u];
    }
    if (lane >= kd && lane < q - 1) {
      L.actid[lane] = id_n; L.actside[lane] = sd_n; L.acte[lane] = e_n; L.actc[lane] = c_n;
      lamr = lam_n;
    }
    bsync<kWS>();
    for (int j = kd; j < q - 1; ++j) {
      const double a = L.Rm[j * NS + j], b = L.Rm[(j + 1) * NS + j];
      const double rr_ = hypot(a, b);
      const double cg = rr_ > 0.0 ? a / rr_ : 1.0, sg = rr_ > 0.0 ? b / rr_ : 0.0;
      double r1 = 0, r2 = 0, qa = 0, qb = 0;
      if (lane >= j && lane < q - 1) { r1 = L.Rm[j * NS + lane]; r2 = L.Rm[(j + 1) * NS + lane]; }
      if (vl) { qa = L.Q1[j * NS + lane]; qb = L.Q1[(j + 1) * NS + lane]; }
      bsync<kWS>();
      if (lane >= j && lane < q - 1) {
        L.Rm[j * NS + lane] = cg * r1 + sg * r2;
        L.Rm[(j + 1) * NS + lane] = -sg * r1 + cg * r2;
      }
      if (vl) {
        L.Q1[j * NS + lane] = cg * qa + sg * qb;
        L.Q1[(j + 1) * NS + lane] = -sg * qa + cg * qb;
      }
      bsync<kWS>();
    }
    --q;
    if (lane >= q) lamr = 0.0;
    if (lane < q) L.Rd[lane] = 1.0 / L.Rm[lane * NS + lane];
    bsync<kWS>();
    ri_rebuild();
  };

  // multipliers of the current working set at the minimiser on its face:
  // R^T w = e_free, R lam = Q1^T v0 - w   (lane k holds entry k)
  auto solve_lambda = [&]() {
    double w = (lane < q) ? (L.acte[lane] - L.actc[lane]) : 0.0;
    for (int k = 0; k < q; ++k) {
      const double wk = wave::bcast(w, k) * L.Rd[k];
      if (lane == k) w = wk;
      else if (lane > k && lane < q) w -= L.Rm[k * NS + lane] * wk;
    }
    if (vl) L.vD[lane] = v0;
    bsync<kWS>();
    double u = 0.0;
    if (lane < q) {
      for (int i = 0; i < N; ++i) u += L.Q1[lane * NS + i] * L.vD[i];
      u -= w;
    }
    for (int k = q - 1; k >= 0; --k) {
      const double lk = wave::bcast(u, k) * L.Rd[k];
      if (lane == k) u = lk;
      else if (lane < k) u -= L.Rm[lane * NS + k] * lk;
    }
    lamr = (lane < q) ? u : 0.0;
    bsync<kWS>();
  };

  // ---- warm start from the ADMM proposal
  const int max_steps = A.max_steps > 0 ? A.max_steps : 8 * N + 64;
  for (int add = 0; kAdmm && add < N; ++add) {
    double best = -1.0;
    int key = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < NFP; ++s)
      if (sc_f[s] > 0.0f && (double(sc_f[s]) > best)) { best = sc_f[s]; key = 2 * (s * nf + lane) + 1; }
    if (sc_d > 0.0f && double(sc_d) > best) { best = sc_d; key = 2 * (F + lane) + (side_d > 0 ? 1 : 0); }
#pragma unroll
    for (int sl = 0; sl < 2; ++sl)
      if (sc_r[sl] > 0.0f && double(sc_r[sl]) > best) { best = sc_r[sl]; key = 2 * (RB + lane + kWave * sl) + 1; }
    wargmax(best, key);
    if (!(best > 0.0) || key < 0 || (key >> 1) >= m) break;
    const int id = key >> 1, side = (key & 1) ? 1 : -1;
    // owner clears its proposal and publishes the full-row bound and constant
    {
      int ol, bit;
      slot_of(id, ol, bit);
      if (lane == ol) {
        if (bit < NFP) {
#pragma unroll
          for (int s = 0; s < NFP; ++s)
            if (s == bit) sc_f[s] = -1.0f;
          L.scal[0] = fu; L.scal[1] = 0.0;
        } else if (bit == NFP) {
          sc_d = -1.0f;
          L.scal[0] = side > 0 ? dbd : -dlo_of(dbd);  // side*bound: u = dbd and -l
          L.scal[1] = double(side) * dcst;
        } else if (bit == NFP + 1) {
          sc_r[0] = -1.0f; L.scal[0] = ru[0]; L.scal[1] = rcst[0];
        } else {
          sc_r[1] = -1.0f; L.scal[0] = ru[1]; L.scal[1] = rcst[1];
        }
      }
    }
    bsync<kWS>();
    const double e_full = L.scal[0], c_full = L.scal[1];
    const double a_own = build_normal(id, side);
    double zz, aa, z_own, r_own, c_own;
    project(a_own, zz, aa, z_own, r_own, c_own);
    if (zz > 1e-16 * aa && q < N) append(sqrt(zz), id, side, e_full, c_full, r_own, z_own, c_own);
  }
  if (q == 0) {
    // no warm start: the unconstrained minimiser
    vw = vl ? v0 : 0.0;
  } else {
    // make the working set dual feasible
    for (int guard = 0; guard <= N; ++guard) {
      solve_lambda();
      double mn = (lane < q) ? lamr : 1.0;
      int kd = lane;
      wargmin(mn, kd);
      if (q == 0 || mn >= 0.0) break;
      drop(kd);
    }
    // v = v0 - Q1 R lam
    if (lane < q) L.vD[lane] = lamr;
    bsync<kWS>();
    if (lane < q) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double rk = L.Rm[lane * NS + k], dk = L.vD[k];
        acc += (k >= lane && k < q) ? rk * dk : 0.0;
      }
      L.vE[lane] = acc;
    }
    bsync<kWS>();
    if (vl) {
      double acc = v0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const double qk = L.Q1[k * NS + lane], ek = L.vE[k];
        acc -= (k < q) ? qk * ek : 0.0;
      }
      vw = acc;
    }
    bsync<kWS>();
  }

  // ---- main loop
  // Evaluate every owned row at the current point (row values to rowval) and
  // return the lane's most violated inactive row as (score, key).
  // Each lane also keeps, for its own best candidate, the violation
  // side * value - e_full and the row's e_full and c_full, which the owning
  // lane hands to the others afterwards (no second evaluation).  The free
  // entries of the point are uniform: they are loaded once, together with
  // the lane's reachable-row coefficients, before any of them is used (the
  // pinned entries of y~ are 0 at P_0 and the goal offset, whose product
  // with a reachable row is the constant rcst).
  auto eval_rows = [&](double& best, int& key, double& sv_b, double& e_b, double& c_b) {
    const int ln = opaque(lane);   // addresses formed here, not held across the loop
    best = -1.0; key = 0x7fffffff; sv_b = 0.0; e_b = 0.0; c_b = 0.0;
    double y[N];
#pragma unroll
    for (int i = 0; i < N; ++i) y[i] = L.ybuf[3 + i];
    // difference rows: lane-dependent entries, branch-free (a velocity lane
    // reads its first entry twice and gives it weight 0)
    const int di0 = 3 * dk + dc, di1 = di0 + 3, di2 = dvel ? di0 : di0 + 6;
    const double yd0 = dl ? L.ybuf[di0] : 0.0, yd1 = dl ? L.ybuf[di1] : 0.0, yd2 = dl ? L.ybuf[di2] : 0.0;
    // reachable row ``lane`` (row 0 stands in on lanes without one)
    double hv[N];
    {
      const double* hr = L.Hd + (ln < r ? ln : 0) * HDS + 3;
#pragma unroll
      for (int i = 0; i < N; ++i) hv[i] = hr[i];
    }
    if (fl) {
#pragma unroll
      for (int s = 0; s < NFP; ++s) {
        const double v = fa0 * y[3 * s] + fa1 * y[3 * s + 1] + fa2 * y[3 * s + 2];
        const int id = s * nf + lane;
        L.rowval[s * nf + ln] = v;
        const double viol = v - fu;
        if (!((act_bits >> s) & 1u) && viol > ftol * (1.0 + fabs(fu))) {
          const double sc = viol * (ifan * K.rkappa[s]);
          if (sc > best) { best = sc; key = 2 * id + 1; sv_b = viol; e_b = fu; c_b = 0.0; }
        }
      }
    }
    if (dl) {
      const double v = dvel ? dsc * (yd1 - yd0) : dsc * (yd2 - 2.0 * yd1 + yd0);
      L.rowval[F + ln] = v;
      if (!((act_bits >> NFP) & 1u)) {
        const double vu = v - dbd, vlo = dlo_of(dbd) - v, dtol = ftol * (1.0 + fabs(dbd));
        if (vu > dtol && vu * ddn > best) { best = vu * ddn; key = 2 * (F + lane) + 1; sv_b = vu; e_b = dbd; c_b = dcst; }
        if (vlo > dtol && vlo * ddn > best) {
          best = vlo * ddn; key = 2 * (F + lane); sv_b = vlo; e_b = -dlo_of(dbd); c_b = -dcst;
        }
      }
    }
    auto reach_row = [&](int sl, const double (&h)[N]) {
      const int l = lane + kWave * sl;
      const int lo = ln + kWave * sl;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < N; ++i) acc += h[i] * y[i];
      const double v = acc + rcst[sl];
      L.rowval[RB + lo] = v;
      const double viol = v - ru[sl];
      if (!((act_bits >> (NFP + 1 + sl)) & 1u) && viol > ftol * (1.0 + fabs(ru[sl]))) {
        const double sc = rdn[sl] > 0.0 ? viol * rdn[sl] : __builtin_huge_val();
        if (sc > best) { best = sc; key = 2 * (RB + l) + 1; sv_b = viol; e_b = ru[sl]; c_b = rcst[sl]; }
      }
    };
    if (lane < r) reach_row(0, hv);
    if (r > kWave) {   // second reachable slot: rows 64..127
      const double* hr = L.Hd + (ln + kWave < r ? ln + kWave : 0) * HDS + 3;
#pragma unroll
      for (int i = 0; i < N; ++i) hv[i] = hr[i];
      if (lane + kWave < r) reach_row(1, hv);
    }
  };
  // x-space point from the whitened one; vD holds vw (written after every
  // update of vw, ahead of a barrier)
  auto refresh_y = [&]() {
    if (vl) L.ybuf[3 + lane] = unwhiten_at<P>(L.cL1i, in.T15, L.vD, lane);
    bsync<kWS>();
  };

  // Dual bound with multipliers lamp >= 0 on the entering row and max(lam, 0)
  // on the working set: for every feasible x, f(x) >= L(x, mu) >= min_x L =
  // c0 - mu'b - 1/2 |L^-1 (q + rho)|^2  (rho = sum mu_k a_k, b the rows'
  // right-hand sides), in whitened form D = 1/2 |v0|^2 - mu'b -
  // 1/2 |L^-1 rho - v0|^2.  D > Uw (every objective value in the box) means
  // no feasible point exists.  Rows and right-hand sides are rebuilt here
  // from the instance data in FP64; the margin covers rounding.
  auto dual_bound_certified = [&](int id, int side, double e_full, double c_full, double lp) -> bool {
    if (lane < q) L.lam[lane] = fmax(lamr, 0.0);
    bsync<kWS>();
    double rx = 0.0;
    if (vl) {
      const int pt = vs + 1;
      rx = lp * double(side) * in.coef(id, pt, vc, L.Af, L.Hd);
      for (int k = 0; k < q; ++k) rx += L.lam[k] * double(L.actside[k]) * in.coef(L.actid[k], pt, vc, L.Af, L.Hd);
    }
    double mb = lp * (e_full - c_full), mbabs = fabs(mb);
    for (int k = 0; k < q; ++k) {
      const double t = L.lam[k] * (L.acte[k] - L.actc[k]);
      mb += t;
      mbabs += fabs(t);
    }
    if (vl) L.vE[lane] = rx;
    bsync<kWS>();
    const double wr = vl ? whiten_at<P>(L.cL1i, in.T15, L.vE, lane) - v0 : 0.0;
    const double hv = 0.5 * wsum(v0 * v0), hr = 0.5 * wsum(wr * wr);
    const double D = hv - mb - hr;
    bsync<kWS>();
    return D > Uw + 1e-9 * (hv + hr + mbabs + Uw) + 1e-12;
  };
  int bound_tries = 0;

  if (vl) L.vD[lane] = vw;
  bsync<kWS>();
  // dual value of the current multipliers (objective 1/2 |v - v0|^2 plus the
  // entering row's multiplier times its violation), carried along the steps:
  // a step of length t adds t (s+ - t zz / 2)
  double dual = q == 0 ? 0.0 : 0.5 * wsum(vl ? (vw - v0) * (vw - v0) : 0.0);
  bool certified_infeasible = false;
  while (true) {
    refresh_y();
    double best, sv_b, e_b, c_b;
    int key;
    eval_rows(best, key, sv_b, e_b, c_b);   // the last pass leaves the solution's row values
    // the largest score; among equal scores the lowest lane's candidate
    const double gbest = wmax(best);
    if (!(gbest > 0.0)) { status = kSolved; break; }
    const int owner = __builtin_ctzll(__ballot(best == gbest));
    key = __builtin_amdgcn_readlane(key, owner);
    if (steps >= max_steps || key < 0 || (key >> 1) >= m) { status = kPolishFailed; break; }
    const int id = key >> 1, side = (key & 1) ? 1 : -1;
    // the owning lane hands over its violation (> 0), full-row bound and
    // constant
    double splus = wave::bcast(sv_b, owner);
    const double e_full = wave::bcast(e_b, owner), c_full = wave::bcast(c_b, owner);
    const double a_own = build_normal(id, side);
    double lamp = 0.0;
    bool added = false;
    while (!added) {
      ++steps;
      double zz, aa, z_own, rv, c_own;   // |z|^2, |a|^2, z_i, r = R^-1 c and c on lanes < q
      project(a_own, zz, aa, z_own, rv, c_own);
      // step to the first multiplier that reaches 0: the smallest lam_k / r_k
      // over r_k > 1e-13 max |r|.  The arg-min over every r_k > 0 and the
      // maximum are reduced together; only when the winner's r_k is below
      // the threshold (rare) is the arg-min taken again over the others.
      double t1 = __builtin_huge_val();
      int kd = lane;
      if (q > 0) {
        double rmax = (lane < q) ? fabs(rv) : 0.0;
        if (lane < q && rv > 0.0) t1 = lamr / rv;
        rmax = wmax(rmax);
        wargmin(t1, kd);
        if (t1 < __builtin_huge_val() && !(wave::bcast(rv, kd) > 1e-13 * rmax)) {
          t1 = __builtin_huge_val();
          kd = lane;
          if (lane < q && rv > 1e-13 * rmax) t1 = lamr / rv;
          wargmin(t1, kd);
        }
      }
      const bool zfull = zz > 1e-20 * aa;
      const double t2 = zfull ? splus / zz : __builtin_huge_val();
      if (!(t1 < 1e300) && !(t2 < 1e300)) {
        // infeasible: Farkas weights 1 on the entering constraint, -r_k >= 0 on the working set
        if (lane < q) L.lam[lane] = fmax(-rv, 0.0);
        bsync<kWS>();
        // residual rho = c+ + sum_k w_k c_k (x-space, free vars) and beta
        double rres = 0.0;
        if (vl) {
          const int pt = vs + 1;
          rres = double(side) * in.coef(id, pt, vc, L.Af, L.Hd);
          for (int k = 0; k < q; ++k)
            rres += L.lam[k] * double(L.actside[k]) * in.coef(L.actid[k], pt, vc, L.Af, L.Hd);
        }
        double beta = (e_full - c_full);
        double wsum_abs = fabs(e_full - c_full);
        for (int k = 0; k < q; ++k) {
          const double ek = L.acte[k] - L.actc[k];
          beta += L.lam[k] * ek;
          wsum_abs += fabs(L.lam[k] * ek);
        }
        // box every feasible x lies in (velocity chain from both pinned ends)
        double lo = 0, hi = 0;
        bool empty = false;
        if (vl) {
          const int k = vs + 1;
          const double vv = in.vmax * in.T / P, dgc = sel3(vc, in.dg[0], in.dg[1], in.dg[2]);
          lo = fmax(-k * vv, dgc - (P - k) * vv);
          hi = fmin(k * vv, dgc + (P - k) * vv);
          empty = lo > hi;
        }
        const double mbox = wsum(vl ? (rres > 0.0 ? rres * lo : rres * hi) : 0.0);
        const bool ok = wany(empty) || (beta < mbox - 1e-12 * (1.0 + wsum_abs));
        certified_infeasible = ok;
        status = ok ? kInfeasible : kPolishFailed;
        break;
      }
      const double t = fmin(t1, t2);
      if (zfull && vl) vw -= t * z_own;
      if (vl) L.vD[lane] = vw;
      if (lane < q) lamr -= t * rv;
      lamp += t;
      dual += t * (splus - 0.5 * t * (zfull ? zz : 0.0));
      if (zfull) splus -= t * zz;
      // once the dual value passes the bound of the objective, try the FP64
      // certificate (which recomputes the dual value from the rows)
      if (bound_tries < 4) {
        if (dual > Uw * (1.0 + 1e-9) + 1e-12) {
          ++bound_tries;
          if (dual_bound_certified(id, side, e_full, c_full, lamp)) {
            certified_infeasible = true;
            status = kInfeasible;
            break;
          }
        }
      }
      if (t2 <= t1) {
        append(sqrt(zz), id, side, e_full, c_full, rv, z_own, c_own);
        if (lane == q - 1) lamr = lamp;
        added = true;
      } else {
        drop(kd);
        if (steps >= max_steps) break;
      }
    }
    if (status == kInfeasible || (status == kPolishFailed && !added)) break;
  }
  (void)certified_infeasible;

  if (status != kSolved) {
    finish_nan(status);
    if (lane == 0 && A.iters_out) { A.iters_out[2 * inst] = K_admm; A.iters_out[2 * inst + 1] = steps; }
    return;
  }

  // ---- solution, KKT residuals, cost
  // ybuf and rowval hold the solution and its row values from the main
  // loop's last pass (no row was violated there).  Every lane forms its
  // partial values first; the reductions then run together.
  bsync<kWS>();
  // primal residual and scale over all rows (owners)
  double pres = 0.0, pscale = 0.0;
  if (fl) {
#pragma unroll
    for (int s = 0; s < NFP; ++s) {
      const double v = L.rowval[s * nf + lane];
      pres = fmax(pres, v - fu);
      pscale = fmax(pscale, fmax(fabs(v), fabs(fu)));
    }
  }
  if (dl) {
    const double v = L.rowval[F + lane];
    pres = fmax(pres, fmax(v - dbd, dlo_of(dbd) - v));
    pscale = fmax(pscale, fmax(fabs(v), fabs(dbd)));
  }
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int l = lane + kWave * sl;
    if (l < r) {
      const double v = L.rowval[RB + l];
      pres = fmax(pres, v - ru[sl]);
      pscale = fmax(pscale, fmax(fabs(v), fabs(ru[sl])));
    }
  }
  // (Q y~)_e for every full coefficient, cost = y~^T Q y~
  double qy = 0.0, yq = 0.0;
  if (lane < NC) {
    const int pt = lane / 3, c = lane - 3 * (lane / 3);
#pragma unroll
    for (int b = 0; b <= P; ++b) qy += L.cQ1[kMaxPts * pt + b] * L.ybuf[3 * b + c];
    qy *= in.iT3;
    L.qbuf[lane] = qy;
    yq = qy * L.ybuf[lane];
  }
  // complementarity
  const double lam_own = fmax(lamr, 0.0);
  double cres = 0.0, lmax = 0.0;
  if (lane < q) {
    L.lam[lane] = lam_own;
    const int id = L.actid[lane];
    const double slack = L.acte[lane] - double(L.actside[lane]) * L.rowval[id];
    cres = lam_own * fabs(slack);
    lmax = lam_own;
  }
  bsync<kWS>();
  // stationarity on the free variables: 2 Q y~ + sum_k lam_k side_k a_k
  // lanes 0..5 also form the multipliers of the pinned coordinates (start
  // point, then goal):  nu = -(2 (Q y~)_pinned + sum_k lam_k side_k a_k,pinned)
  double st = 0.0, sq = 0.0, sac = 0.0, spin = 0.0;
  const int ppt = lane < 3 ? 0 : P, pc = lane - 3 * (lane / 3);
  // row k's id and signed multiplier from lane k's registers (no LDS round
  // trip per row)
  const int id_r = lane < q ? L.actid[lane] : 0;
  const double ls_r = lane < q ? lam_own * double(L.actside[lane]) : 0.0;
  if (vl) {
    const int pt = vs + 1;
    sq = 2.0 * L.qbuf[3 + lane];
    for (int k = 0; k < q; ++k) {
      const int idk = __builtin_amdgcn_readlane(id_r, k);
      const double ls = wave::bcast(ls_r, k);
      sac += ls * in.coef(idk, pt, vc, L.Af, L.Hd);
      if (A.store) spin += ls * in.coef(idk, ppt, pc, L.Af, L.Hd);
    }
    st = sq + sac;
  }
  if (A.store && lane < 6) A.fw_nu[6 * (int64_t)inst + lane] = -(2.0 * L.qbuf[3 * ppt + pc] + spin);
  pres = wmax(pres);
  pscale = wmax(pscale);
  const double cost = wsum(yq);
  const double stm = wmax(fabs(st)), sqm = wmax(fabs(sq)), sacm = wmax(fabs(sac));
  lmax = wmax(lmax);
  cres = wmax(cres);
  const double dres = stm / (1.0 + fmax(sqm, sacm));
  cres = cres / (1.0 + lmax);
  const double kkt = fmax(fmax(fmax(pres, 0.0) / (1.0 + pscale), dres), cres);
  const bool ok = kkt <= A.kkt_tol && isfinite(kkt) && isfinite(cost);
  if (lane < NC) {
    const double pv = L.ybuf[lane] + sel3(lane - 3 * (lane / 3), in.P0[0], in.P0[1], in.P0[2]);
    A.P_out[3 * in.po + lane] = pv;
  }
  if (lane == 0) {
    A.cost_out[inst] = cost;
    A.status_out[inst] = ok ? kSolved : kNumerical;
    if (A.store) A.fw_status[inst] = ok ? kSolved : kNumerical;
    A.kkt_out[inst] = kkt;
    if (A.iters_out) { A.iters_out[2 * inst] = K_admm; A.iters_out[2 * inst + 1] = steps; }
    if (A.store) A.st_q[inst] = q;
  }
  if (A.store && lane < q) {
    const int64_t b = (int64_t)inst * A.st_stride;
    A.st_id[b + lane] = L.actid[lane];
    A.st_side[b + lane] = L.actside[lane];
    A.st_lam[b + lane] = L.lam[lane];
  }
  // the factor of the final working set for the backward pass, packed:
  // rows k < q of Q1 (N entries each), then the q x q block of R (upper
  // triangle written), element-parallel
  if (A.store) {
    constexpr int EPL = (N * N + kWave - 1) / kWave;
    const int S = A.st_stride;
    double* qr = A.st_qr + (int64_t)inst * 2 * S * S;
    const int ln = opaque(lane);
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      const int e = ln + kWave * u;
      const int k = e / N, i = e - N * (e / N);
      if (k < q) {
        qr[k * N + i] = L.Q1[k * NS + i];
        if (i >= k && i < q) qr[q * N + k * q + i] = L.Rm[k * NS + i];
      }
    }
  }
}

// ==========================================================================
// Backward pass: implicit differentiation of the KKT system on the stored
// active set.  For loss  l = gP . P* + gf * f*:
//   [2Q_ff  C^T; C 0] [w; omega] = [gP_free; 0]   (C: active rows, side-signed)
//   omega_E = gP_pinned - 2 Q_{pinned,free} w - C_pinned^T omega
//   nu      = -(2 (Q y~)_pinned + C_pinned^T lam)
//   d l / d b_j  = sum over active face rows on face j of (omega - gf lam)
//   d l / d x0   = G^T (omega - gf lam)_reach + [(omega_E - gf nu)_start; 0]
//   d l / d goal = (omega_E - gf nu)_goal
// ==========================================================================
template <int P>
__device__ void backward_instance(const BackArgs& A, const InstDesc& idesc, char* smem) {
  using I = Inst<P>;
  constexpr int NFP = I::NFP, N = I::N, NC = I::NC, ND = I::ND, NS = I::NS;
  const int lane = threadIdx.x;
  const DegConst& K = c_deg[P];
  const LdsDims& D = A.dims;
  Lds<double> L = carve<double>(smem, D);
  const int inst = idesc.inst;
  I in;
  in.T = A.T[inst];
  in.f0 = idesc.f0;
  in.nf = idesc.nf;
  in.r0 = idesc.r0;
  in.r = idesc.r;
  in.hb = idesc.hb;
  in.po = idesc.po;
  in.F = NFP * in.nf;
  in.RB = in.F + ND;
  in.m = in.RB + in.r;
  in.T15 = in.T * sqrt(in.T);
  in.iT3 = 1.0 / (in.T * in.T * in.T);
  in.sv = double(P) / in.T;
  in.sa = double(P) * (P - 1) / (in.T * in.T);
  const int64_t fo = idesc.fo;
  const int nf = in.nf, r = in.r;
  // every global load of the prologue depends only on the descriptor: all
  // are issued before the first wait (the stored active set is read on
  // every lane below its stride, whatever q turns out to be)
  const int64_t sb = (int64_t)inst * A.st_stride;
  const int st = A.status[inst];
  const int qs = A.st_q[inst];
  int sid = 0, sside = 0;
  double slam = 0.0;
  if (lane < A.st_stride) { sid = A.st_id[sb + lane]; sside = A.st_side[sb + lane]; slam = A.st_lam[sb + lane]; }
  const double nu = lane < 6 ? A.nu[6 * (int64_t)inst + lane] : 0.0;
  const double gpv = (lane < NC && A.grad_P) ? A.grad_P[3 * in.po + lane] : 0.0;
  const double gf = A.grad_cost ? A.grad_cost[inst] : 0.0;
  const int q = st == kSolved ? qs : -1;
  if (q < 0) {
    if (lane < 6) A.grad_x0[6 * (int64_t)inst + lane] = 0.0;
    if (lane < 3) A.grad_goal[3 * (int64_t)inst + lane] = 0.0;
    for (int j = lane; j < nf; j += kWave) A.grad_b[fo + j] = 0.0;
    if (A.flags && lane == 0) A.flags[inst] = 0;
    return;
  }
  if (A.debug_fill) {   // debug option: poison the LDS first (see the forward pass)
    double* w = reinterpret_cast<double*>(smem);
    for (int e = lane; e < D.bytes / 8; e += kWave) w[e] = __builtin_nan("");
    __syncthreads();
  }
  for (int e = lane; e < nf * 3; e += kWave) L.Af[e] = A.A_face[3 * (int64_t)in.f0 + e];
  for (int e = lane; e < kMaxFree * kMaxFree; e += kWave) L.cL1i[e] = (&K.L1inv[0][0])[e];
  if (lane < q) {
    L.actid[lane] = sid;
    L.actside[lane] = sside;
    L.lam[lane] = slam;
  }
  // upstream gradient on the full control points -> qbuf (reused)
  if (lane < NC) L.qbuf[lane] = gpv;
  // the adjoint needs the active reachable rows only on the pinned points
  // (their coefficients on P_0 and P_p): six entries per row, packed by
  // working-set slot (Hd[6 k + j]); the row id of active row k comes from
  // lane k's register
  for (int base = 0; base < q * 6; base += 2 * kWave) {
    double v[2];
    int dst[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = base + u * kWave + lane;
      const bool live = t < q * 6;
      const int k = live ? t / 6 : 0, j = t - 6 * (t / 6);
      const int e = j < 3 ? j : 3 * P + j - 3;
      const int idk = __shfl(sid, k, kWave);
      const int id = live ? idk : -1;
      const bool take = id >= in.RB;
      dst[u] = take ? 6 * k + j : -1;
      v[u] = take ? A.H[in.hb + (int64_t)(id - in.RB) * NC + e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
      if (dst[u] >= 0) L.Hd[dst[u]] = v[u];
  }
  // the factor of the final working set (packed by the forward pass: rows
  // k < q of Q1, then the q x q block of R)
  {
    constexpr int EPL = (N * N + kWave - 1) / kWave;
    const int S = A.st_stride;
    const double* qr = A.st_qr + (int64_t)inst * 2 * S * S;
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      const int e = lane + kWave * u;
      const int k = e / N, i = e - N * (e / N);
      if (k < q) {
        L.Q1[k * NS + i] = qr[k * N + i];
        if (i >= k && i < q) L.Rm[k * NS + i] = qr[q * N + k * q + i];
      }
    }
  }
  __syncthreads();
  const bool vl = lane < N;
  const int vs = lane / 3, vc = lane - 3 * (lane / 3);
  // the factor of the active normals (whitened, in stored order), kept by
  // the forward pass; a diagonal entry near 0 flags dependent active rows
  const bool dep = wany(lane < q && !(L.Rm[lane * NS + lane] > 1e-10));
  // whitened upstream gradient on the free variables
  if (vl) L.vD[lane] = L.qbuf[3 + lane];
  __syncthreads();
  double gh = vl ? whiten_at<P>(L.cL1i, in.T15, L.vD, lane) : 0.0;
  if (vl) L.vA[lane] = gh;
  __syncthreads();
  // c = Q1^T gh ; omega = R^-1 c ; xi = gh - Q1 c ; w = L^-T xi
  const double cv = lane < q ? dot_row<N>(L.Q1 + lane * NS, L.vA) : 0.0;
  if (lane < q) L.vE[lane] = cv;
  __syncthreads();
  double om = cv;
  for (int k = q - 1; k >= 0; --k) {
    const double ok = wave::bcast(om, k) / L.Rm[k * NS + k];
    if (lane == k) om = ok;
    else if (lane < k) om -= L.Rm[lane * NS + k] * ok;
  }
  if (vl) L.vB[lane] = colsub_q(gh, L.Q1 + lane, NS, L.vE, q);
  __syncthreads();
  if (vl) L.vC[lane] = unwhiten_at<P>(L.cL1i, in.T15, L.vB, lane);   // w on the free vars
  // combined row weights  Omega_k = omega_k - gf lam_k
  if (lane < q) L.vD[lane] = om - gf * L.lam[lane];
  __syncthreads();
  // pinned rows: omega_E per coordinate (lanes 0..5: e = start c / goal c);
  // nu of the same coordinate was formed by the forward pass
  if (lane < 6) {
    const int c = lane % 3;
    const int pt = lane < 3 ? 0 : P;
    // (2 Q)_{pt, free} w
    double qw = 0.0;
    for (int s = 0; s < NFP; ++s) qw += K.Q1[pt][s + 1] * L.vC[3 * s + c];
    qw *= 2.0 * in.iT3;
    double cw = 0.0;
    for (int k = 0; k < q; ++k) {
      const int idk = L.actid[k];
      const double a = double(L.actside[k]) *
                       (idk >= in.RB ? L.Hd[6 * k + (pt == 0 ? c : 3 + c)] : in.coef(idk, pt, c, L.Af, L.Hd));
      cw += a * (L.vD[k] + gf * L.lam[k]);   // omega_k
    }
    const double omE = L.qbuf[3 * pt + c] - qw - cw;
    L.scal[lane] = omE - gf * nu;
  }
  __syncthreads();
  // gradients
  if (lane < 6) {
    double g = (lane < 3) ? L.scal[lane] : 0.0;
    for (int k = 0; k < q; ++k) {
      const int id = L.actid[k];
      if (id >= in.RB) g += L.vD[k] * A.G[6 * (in.r0 + (id - in.RB)) + lane];
      // pinned start velocity: row F + c bounds its value by x0[3+c] on the
      // active side (right-hand side side * x0[3+c])
      if (A.pin_v0 && lane >= 3 && id == in.F + lane - 3) g += L.vD[k] * double(L.actside[k]);
    }
    A.grad_x0[6 * (int64_t)inst + lane] = g;
  }
  if (lane < 3) A.grad_goal[3 * (int64_t)inst + lane] = L.scal[3 + lane];
  for (int j = lane; j < nf; j += kWave) {
    double g = 0.0;
    for (int k = 0; k < q; ++k) {
      const int id = L.actid[k];
      if (id < in.F && (id - (id / nf) * nf) == j) g += L.vD[k];
    }
    A.grad_b[fo + j] = g;
  }
  if (A.flags && lane == 0) A.flags[inst] = dep ? 1 : 0;
}

}  // namespace
}  // namespace rbp
