// Batched MPC refinement QP (eq. MPC, Sec. III-D): one 64-lane wave per
// instance, primal-dual interior point (Mehrotra predictor-corrector), FP64.
//
// Stage variables z_k = (x_k, u_k), k = 0..N-1, with x = (position, velocity)
// and u = acceleration; x_{k+1} = A x_k + B u_k is the exact discretisation of
// the double integrator over dt.  x_0 = x0 and x_N = r_N are fixed.  Stage
// cost 1/2 z'H z + h'z with h_k = (-2 Q r_k, 0) (no tracking at k = 0), so
// the cost of the problem is the sum plus the constants r_k'Q r_k.  Rows of
// stage k, each scaled to unit norm, c_i'z_k <= d_i: the m reachable rows
// F1 x_k + F2 x_{k+1} <= G (Thm. 2) with x_{k+1} substituted, then four
// keep-out rows n_k . P_j >= l_k on the control points of the cubic that
// joins the two states (Lemma 1), P_j = p + a_j v + b_j u.
//
// Every Newton system is an equality-constrained LQ problem:
//   min sum_k 1/2 dz_k' Ht_k dz_k + g_k' dz_k,  dynamics, dx_0 = 0, dx_N = 0,
// with Ht_k = H_k + sum_i (lam_i / s_i) c_i c_i'.  It is solved by a Riccati
// recursion in Cholesky form (Quu = L L', Y = L^-1 Qux, P = Qxx - Y'Y) with
// the cost-to-go symmetrised at every stage: the plain update
// P = Qxx - Qxu Quu^-1 Qux drifts away from symmetry and loses all accuracy
// once some barrier weights are large.  The terminal state is fixed by
// eliminating the last two stages exactly: [u_{N-2}; u_{N-1}] =
// [AB B]^-1 (-A^2 x_{N-2}), so z_{N-2} = T2 x_{N-2} and z_{N-1} = T1 x_{N-2}.
//
// The dual residual is not carried along: every iteration fits the costates
// (x-stationarity fixes pi_k from pi_{k+1}; pi_N is chosen by least squares)
// and feeds the remaining u-stationarity residual into the Newton system, so
// errors of earlier directions do not accumulate.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "rbp_internal.hpp"
#include "rbp_wave.hpp"

namespace rbp {
namespace {

constexpr int kW = 64;
constexpr int kSolved = 0, kInfeasible = 1, kMaxIter = 2, kNumerical = 4, kInvalid = 5;

// LDS carve, in doubles.  The per-row state (slack, multiplier, primal
// residual, Newton weight) lives in registers of the lane that owns the row;
// LDS holds one value per row, X, for the reads that cross lanes: the
// multipliers (dual residual), the barrier weights lam/s (factorisation), the
// Newton weights (gradient build), and meanwhile each row's c'dz for its own
// lane.  The gradient of the LQ solve shares its storage with the direction
// it produces.
struct MpcSm {
  double *prm, *z, *g, *dz, *ref, *pl, *X, *Lc, *Y, *yv, *rho, *P, *tmp;
  // scratch of the factorisation, inside the gradient buffer (free while it runs)
  double *Ht, *Qh, *HtT;
};

// the gradient / direction buffer also holds the factorisation's scratch
// (Ht 81, Qh 81, Ht T 54)
__host__ __device__ inline int mpc_g_doubles(int N) { return 9 * N > 288 ? 9 * N : 288; }

__host__ __device__ inline int mpc_lds_doubles(int N, int m) {
  const MpcLayout L = mpc_param_layout(m);
  const int RT = N * (m + 4);
  return L.total + 9 * N /*z*/ + mpc_g_doubles(N) /*g = dz*/ + 6 * (N + 1) /*ref*/ + 4 * N /*pl*/ +
         RT /*X*/ + 6 * N /*Lc*/ + 18 * N /*Y*/ + 3 * N /*yv*/ + 3 * N /*rho*/ + 36 /*P*/ + 16 /*tmp*/;
}

__device__ inline MpcSm carve_mpc(double* base, int N, int m) {
  const MpcLayout L = mpc_param_layout(m);
  const int RT = N * (m + 4);
  MpcSm S;
  double* p = base;
  S.prm = p; p += L.total;
  S.z = p; p += 9 * N;
  S.g = p; S.dz = p;
  S.Ht = p; S.Qh = p + 81; S.HtT = p + 162;
  p += mpc_g_doubles(N);
  S.ref = p; p += 6 * (N + 1);
  S.pl = p; p += 4 * N;
  S.X = p; p += RT;
  S.Lc = p; p += 6 * N;
  S.Y = p; p += 18 * N;
  S.yv = p; p += 3 * N;
  S.rho = p; p += 3 * N;
  S.P = p; p += 36;
  S.tmp = p;
  return S;
}

// tmp layout: [0, 6) start state, [8] factorisation flag
constexpr int kTmpFlag = 8;

// Column b of [A B] (6 x 9) has at most two non-zeros: row q0 with weight w0
// and row q1 with weight w1 (q1 < 0: none).
__device__ inline void ab_col(int b, double dt, int& q0, double& w0, int& q1, double& w1) {
  if (b < 3) { q0 = b; w0 = 1.0; q1 = -1; w1 = 0.0; }
  else if (b < 6) { q0 = b; w0 = 1.0; q1 = b - 3; w1 = dt; }
  else { q0 = b - 3; w0 = dt; q1 = b - 6; w1 = 0.5 * dt * dt; }
}

// 1/sqrt(x) and a / b from the hardware approximations (v_rsq_f64, v_rcp_f64)
// refined by Newton steps to full double precision: the chains of a
// factorisation stage and the per-row weights stay short.  x, b > 0 here
// (a non-positive pivot is caught by the caller).
__device__ inline double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  r = r * fma(-hx * r, r, 1.5);
  r = r * fma(-hx * r, r, 1.5);
  return r;
}
__device__ inline double div_nr(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(fma(-b, r, 1.0), r, r);
  r = fma(fma(-b, r, 1.0), r, r);
  const double q = a * r;
  return fma(fma(-b, q, a), r, q);
}

struct MpcCtx {
  const MpcArgs& A;
  MpcSm S;
  MpcLayout Ly;
  int N, m, mr, RT, lane;
  double dt;
  int ua, ub;          // upper-triangle entry (ua <= ub) of a 9 x 9 matrix owned by lanes < 45

  // component a of C_k' w for per-row weights w (rows of stage k at w[0..mr))
  __device__ __forceinline__ double ct_times(int k, int a, const double* w) const {
    const double* c = S.prm + Ly.Cr + a * Ly.cs;
    double t = 0.0, t1 = 0.0;
    int i = 0;
    for (; i + 8 <= m; i += 8) {         // loads of eight rows issued together
      double x[8], y[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) { x[q] = c[i + q]; y[q] = w[i + q]; }
#pragma unroll
      for (int q = 0; q < 8; q += 2) {
        t += x[q] * y[q];
        t1 += x[q + 1] * y[q + 1];
      }
    }
    for (; i < m; ++i) t += c[i] * w[i];
    t += t1;
    const double* f = S.prm + Ly.pf + a / 3;
    const double tp = f[0] * w[m] + f[3] * w[m + 1] + f[6] * w[m + 2] + f[9] * w[m + 3];
    return t - S.pl[4 * k + a % 3] * tp;
  }
  __device__ __forceinline__ const double* Hk(int k) const { return S.prm + (k == 0 ? Ly.H0 : Ly.H1); }
  // x-part of h_k: -2 Q r_k (k >= 1)
  __device__ __forceinline__ double hk(int k, int a) const {
    if (k == 0 || a >= 6) return 0.0;
    double v = 0.0;
    for (int b = 0; b < 6; ++b) v += S.prm[Ly.Qm + 6 * a + b] * S.ref[6 * k + b];
    return -2.0 * v;
  }

  // upper entry (ua, ub) of Ht_k = H_k + sum_i sigma_i c_i c_i', with the
  // barrier weights sigma of stage k's rows in S.X
  __device__ __forceinline__ double ht_entry(int k) const {
    const double* sg = S.X + k * mr;
    const double* ca = S.prm + Ly.Cr + ua * Ly.cs;
    const double* cb = S.prm + Ly.Cr + ub * Ly.cs;
    // the operands outside the row loop are loaded first, so they are in
    // flight together with the first rows
    const double* fa = S.prm + Ly.pf + ua / 3;
    const double* fb = S.prm + Ly.pf + ub / 3;
    const double hv = Hk(k)[9 * ua + ub];
    const double s0 = sg[m], s1 = sg[m + 1], s2 = sg[m + 2], s3 = sg[m + 3];
    const double fa0 = fa[0], fa3 = fa[3], fa6 = fa[6], fa9 = fa[9];
    const double fb0 = fb[0], fb3 = fb[3], fb6 = fb[6], fb9 = fb[9];
    const double pla = S.pl[4 * k + ua % 3], plb = S.pl[4 * k + ub % 3];
    double v = hv, v1 = 0.0;
    int i = 0;
    for (; i + 8 <= m; i += 8) {         // loads of eight rows issued together
      double w[8], x[8], y[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) { w[q] = sg[i + q]; x[q] = ca[i + q]; y[q] = cb[i + q]; }
#pragma unroll
      for (int q = 0; q < 8; q += 2) {
        v += w[q] * x[q] * y[q];
        v1 += w[q + 1] * x[q + 1] * y[q + 1];
      }
    }
    for (; i < m; ++i) v += sg[i] * ca[i] * cb[i];
    v += v1;
    const double tp = s0 * fa0 * fb0 + s1 * fa3 * fb3 + s2 * fa6 * fb6 + s3 * fa9 * fb9;
    return v + pla * plb * tp;
  }

  // Riccati factorisation of the Newton LQ with the barrier weights in S.X
  // (zero weights: H_k alone).  Returns false (uniformly) when a pivot of
  // some Quu is not positive.
  __device__ __forceinline__ bool factor() {
    if (lane == 0) S.tmp[kTmpFlag] = 0.0;
    // terminal block: P = T2' Ht_{N-2} T2 + T1' Ht_{N-1} T1
    for (int e = lane; e < 36; e += kW) S.P[e] = 0.0;
    for (int t = 0; t < 2; ++t) {
      const int k = N - 2 + t;
      const double* T = S.prm + (t == 0 ? Ly.T2 : Ly.T1);
      if (lane < 45) {
        const double v = ht_entry(k);
        S.Ht[9 * ua + ub] = v;
        S.Ht[9 * ub + ua] = v;
      }
      __syncthreads();
      // Ht T (9 x 6)
      for (int e = lane; e < 54; e += kW) {
        const int a = e / 6, c = e - 6 * (e / 6);
        double v = 0.0;
        for (int b = 0; b < 9; ++b) v += S.Ht[9 * a + b] * T[6 * b + c];
        S.HtT[e] = v;
      }
      __syncthreads();
      for (int e = lane; e < 36; e += kW) {
        const int c = e / 6, d = e - 6 * (e / 6);
        double v = 0.0;
        for (int a = 0; a < 9; ++a) v += T[6 * a + c] * S.HtT[6 * a + d];
        S.P[e] += v;
      }
      __syncthreads();
    }
    for (int e = lane; e < 36; e += kW) {
      const int a = e / 6, b = e - 6 * (e / 6);
      if (a < b) {
        const double v = 0.5 * (S.P[e] + S.P[6 * b + a]);
        S.P[e] = v; S.P[6 * b + a] = v;
      }
    }
    __syncthreads();
    for (int k = N - 3; k >= 0; --k) {
      // Qh = Ht + [A B]' P [A B] (symmetric: lanes own the upper triangle)
      if (lane < 45) {
        int qa0, qa1, qb0, qb1;
        double wa0, wa1, wb0, wb1;
        ab_col(ua, dt, qa0, wa0, qa1, wa1);
        ab_col(ub, dt, qb0, wb0, qb1, wb1);
        // absent second terms have weight 0 (ab_col): their loads use a
        // valid entry instead of a branch, so all four are issued together
        const int qa1c = qa1 >= 0 ? qa1 : qa0, qb1c = qb1 >= 0 ? qb1 : qb0;
        const double p00 = S.P[6 * qa0 + qb0], p01 = S.P[6 * qa0 + qb1c];
        const double p10 = S.P[6 * qa1c + qb0], p11 = S.P[6 * qa1c + qb1c];
        double v = wa0 * wb0 * p00;
        v += wa0 * wb1 * p01;
        v += wa1 * wb0 * p10;
        v += wa1 * wb1 * p11;
        v += ht_entry(k);
        S.Qh[9 * ua + ub] = v;
        S.Qh[9 * ub + ua] = v;
      }
      __syncthreads();
      // Quu = L L' and the columns of Y = L^-1 Qux that entry (a, b) of the
      // next cost-to-go P = Qxx - Y'Y needs, all in the lane of that entry
      // (lanes < 21); lanes 0..5 (entries (0, c)) store column c of Y, lane 0
      // stores L as (1/l00, l10, 1/l11, l20, l21, 1/l22).
      if (lane < 21) {
        int a = 0, t = lane;
        while (t >= 6 - a) { t -= 6 - a; ++a; }
        const int b = a + t;
        // every entry this lane reads, loaded before the pivot chain starts
        const double q60 = S.Qh[60], q69 = S.Qh[69], q78 = S.Qh[78], q70 = S.Qh[70], q79 = S.Qh[79],
                     q80 = S.Qh[80];
        const double qa0 = S.Qh[54 + a], qa1 = S.Qh[63 + a], qa2 = S.Qh[72 + a];
        const double qb0 = S.Qh[54 + b], qb1 = S.Qh[63 + b], qb2 = S.Qh[72 + b];
        const double qab = S.Qh[9 * a + b];
        const double d0 = q60;
        const double i00 = rsqrt_nr(d0);
        const double l10 = q69 * i00, l20 = q78 * i00;
        const double d1 = q70 - l10 * l10;
        const double i11 = rsqrt_nr(d1);
        const double l21 = (q79 - l20 * l10) * i11;
        const double d2 = q80 - l20 * l20 - l21 * l21;
        const double i22 = rsqrt_nr(d2);
        const double ya0 = qa0 * i00;
        const double ya1 = (qa1 - l10 * ya0) * i11;
        const double ya2 = (qa2 - l20 * ya0 - l21 * ya1) * i22;
        const double yb0 = qb0 * i00;
        const double yb1 = (qb1 - l10 * yb0) * i11;
        const double yb2 = (qb2 - l20 * yb0 - l21 * yb1) * i22;
        if (lane < 6) {
          double* Y = S.Y + 18 * k;
          Y[b] = yb0; Y[6 + b] = yb1; Y[12 + b] = yb2;
        }
        if (lane == 0) {
          double* L = S.Lc + 6 * k;
          L[0] = i00; L[1] = l10; L[2] = i11; L[3] = l20; L[4] = l21; L[5] = i22;
          if (!(d0 > 0.0 && d1 > 0.0 && d2 > 0.0) || !isfinite(i00 * i11 * i22)) S.tmp[kTmpFlag] = 1.0;
        }
        if (k > 0) {
          const double v = qab - (ya0 * yb0 + ya1 * yb1 + ya2 * yb2);
          S.P[6 * a + b] = v;
          S.P[6 * b + a] = v;
        }
      }
      __syncthreads();
    }
    return S.tmp[kTmpFlag] == 0.0;
  }

  // Solve the factorised LQ for the gradients in S.g; the direction replaces
  // them (S.dz aliases S.g: the backward sweep reads every g_k before the
  // forward sweep writes dz_k).  Sequential over stages in lane 0.
  __device__ __forceinline__ void lq_solve() {
    const double* T2 = S.prm + Ly.T2;
    const double* T1 = S.prm + Ly.T1;
    const double h2 = 0.5 * dt * dt;
    // backward sweep, one costate component per lane: lane c < 6 holds p_c;
    // the u-part of [A B]'p needs p_{c+3} and the x-part p_{c-3}, both a DPP
    // row shift by three lanes away, and y = L^-1 qu takes qu from lanes 0..2
    {
      const int c = lane < 6 ? lane : 5;
      const int cu = lane < 3 ? lane : 2;
      double pc = 0.0;
      for (int a = 0; a < 9; ++a) pc += T2[6 * a + c] * S.g[9 * (N - 2) + a] + T1[6 * a + c] * S.g[9 * (N - 1) + a];
      for (int k = N - 3; k >= 0; --k) {
        const double gx = S.g[9 * k + c], gu = S.g[9 * k + 6 + cu];
        const double Y0 = S.Y[18 * k + c], Y1 = S.Y[18 * k + 6 + c], Y2 = S.Y[18 * k + 12 + c];
        double L[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) L[e] = S.Lc[6 * k + e];
        const double p_up = wave::dpp_f64<0x103>(pc);     // p_{c+3}
        const double p_dn = wave::dpp_f64<0x113>(pc);     // p_{c-3}
        // qh = g + [A B]' p
        const double qx = lane < 3 ? gx + pc : gx + dt * p_dn + pc;
        const double qu = gu + h2 * pc + dt * p_up;
        const double qu0 = wave::bcast(qu, 0), qu1 = wave::bcast(qu, 1), qu2 = wave::bcast(qu, 2);
        const double y0 = qu0 * L[0];
        const double y1 = (qu1 - L[1] * y0) * L[2];
        const double y2 = (qu2 - L[3] * y0 - L[4] * y1) * L[5];
        if (lane < 3) S.yv[3 * k + lane] = lane == 0 ? y0 : (lane == 1 ? y1 : y2);
        pc = qx - (Y0 * y0 + Y1 * y1 + Y2 * y2);
      }
    }
    __syncthreads();
    if (lane == 0) {
      // forward from dx_0 = 0: du = -L^-T (Y dx + y)
      double dx[6] = {0, 0, 0, 0, 0, 0};
      for (int k = 0; k <= N - 3; ++k) {
        double L[6], Y[18], yk[3];
#pragma unroll
        for (int e = 0; e < 6; ++e) L[e] = S.Lc[6 * k + e];
#pragma unroll
        for (int e = 0; e < 18; ++e) Y[e] = S.Y[18 * k + e];
#pragma unroll
        for (int e = 0; e < 3; ++e) yk[e] = S.yv[3 * k + e];
        double r[3];
        for (int i = 0; i < 3; ++i) {
          double v = yk[i];
          for (int c = 0; c < 6; ++c) v += Y[6 * i + c] * dx[c];
          r[i] = v;
        }
        const double u2 = -r[2] * L[5];
        const double u1 = -(r[1] + L[4] * u2) * L[2];
        const double u0 = -(r[0] + L[1] * u1 + L[3] * u2) * L[0];
        double* d = S.dz + 9 * k;
        for (int c = 0; c < 6; ++c) d[c] = dx[c];
        d[6] = u0; d[7] = u1; d[8] = u2;
        const double uu[3] = {u0, u1, u2};
        for (int c = 0; c < 3; ++c) {
          const double pn = dx[c] + dt * dx[3 + c] + h2 * uu[c];
          dx[3 + c] = dx[3 + c] + dt * uu[c];
          dx[c] = pn;
        }
      }
      for (int a = 0; a < 9; ++a) {
        double v2 = 0.0, v1 = 0.0;
        for (int c = 0; c < 6; ++c) { v2 += T2[6 * a + c] * dx[c]; v1 += T1[6 * a + c] * dx[c]; }
        S.dz[9 * (N - 2) + a] = v2;
        S.dz[9 * (N - 1) + a] = v1;
      }
    }
    __syncthreads();
  }

  // visit every row: f(slot, r, c'z_k, c'dz_k, d_r) -- the reachable rows
  // (shared coefficient table), then the plane rows, so a wavefront never
  // mixes the two kinds.  Lane l owns reachable row t = l + 64 j in register
  // slot j < RS and plane row l + 64 j in slot RS + j (j < 4): the loops are
  // unrolled, so slot is a constant wherever f indexes a register array with
  // it.  c'z and c'dz are formed only when CZ / CD ask for them.
  template <int RS, bool CZ, bool CD, typename F>
  __device__ __forceinline__ void for_rows(F&& f) const {
    // the lane index is made opaque here, so the per-slot row indices and
    // addresses are recomputed in every pass instead of being hoisted out of
    // the iteration loop (where they would hold registers throughout)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    if (m > 0) {
      const int rq = kW / m, rr = kW - rq * m;
      int k = ln / m, i = ln - m * (ln / m);
#pragma unroll
      for (int j = 0; j < RS; ++j) {
        if (ln + kW * j < N * m) {
          const double* c = S.prm + Ly.Cr + i;
          const double* zk = S.z + 9 * k;
          const double* dk = S.dz + 9 * k;
          double cz = 0.0, cd = 0.0;
#pragma unroll
          for (int a = 0; a < 9; ++a) {
            const double ca = c[a * Ly.cs];
            if (CZ) cz += ca * zk[a];
            if (CD) cd += ca * dk[a];
          }
          f(j, k * mr + i, cz, cd, S.prm[Ly.dr + i]);
        }
        k += rq;
        i += rr;
        if (i >= m) { i -= m; ++k; }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int t = ln + kW * j;
      if (t < 4 * N) {
        const int k = t >> 2, jj = t & 3;
        const double* f3 = S.prm + Ly.pf + 3 * jj;
        const double* n = S.pl + 4 * k;
        const double* zk = S.z + 9 * k;
        const double* dk = S.dz + 9 * k;
        double cz = 0.0, cd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (CZ) cz += n[c] * (f3[0] * zk[c] + f3[1] * zk[3 + c] + f3[2] * zk[6 + c]);
          if (CD) cd += n[c] * (f3[0] * dk[c] + f3[1] * dk[3 + c] + f3[2] * dk[6 + c]);
        }
        f(RS + j, k * mr + m + jj, -cz, -cd, -n[3] * f3[0]);
      }
    }
  }

  // g_k = [0; rho_k] + C_k' w, with the per-row weights in S.X
  __device__ __forceinline__ void build_g() {
    for (int e = lane; e < 9 * N; e += kW) {
      const int k = e / 9, a = e - 9 * (e / 9);
      const double v = a >= 6 ? S.rho[3 * k + a - 6] : 0.0;
      S.g[e] = v + ct_times(k, a, S.X + k * mr);
    }
    __syncthreads();
  }

  // least-squares costates and the u-stationarity residual rho_k (into
  // S.rho), with the multipliers in S.X; returns max |rho| and the scale of
  // the gradient terms.  kCost = false leaves the cost out: rho is then the
  // gradient in the inputs of sum_i w_i c_i'z + pi'x_N along trajectories of
  // the dynamics from x0, with the terminal costate pi (returned in pi6 when
  // given) chosen by least squares.
  template <bool kCost = true>
  __device__ __forceinline__ void dual_residual(double& rmax, double& gscale, double* pi6 = nullptr) {
    double gs = 0.0;
    for (int e = lane; e < 9 * N; e += kW) {
      const int k = e / 9, a = e - 9 * (e / 9);
      double hz = 0.0;
      if constexpr (kCost) {
        const double* H = Hk(k);
        hz = hk(k, a);
        for (int b = 0; b < 9; ++b) hz += H[9 * a + b] * S.z[9 * k + b];
      }
      const double ct = ct_times(k, a, S.X + k * mr);
      S.g[e] = hz + ct;
      gs = fmax(gs, fmax(fabs(hz), fabs(ct)));
    }
    gscale = wave::max(gs);
    __syncthreads();
    // backward: f_k = e_k + B' sig_{k+1};  sig_k = c_k + A' sig_{k+1} (k >= 1).
    // The axes do not mix: lane c < 3 carries (sig_p,c, sig_v,c), with each
    // stage's three gradient entries loaded two stages ahead
    if (lane < 3) {
      const int c = lane;
      const double h2 = 0.5 * dt * dt;
      double sp_ = 0.0, sv_ = 0.0;
      auto fetch = [&](int k, double& gp, double& gv, double& gu) {
        const int kc = k < 0 ? 0 : k;
        gp = S.g[9 * kc + c]; gv = S.g[9 * kc + 3 + c]; gu = S.g[9 * kc + 6 + c];
      };
      auto stage = [&](int k, double gp, double gv, double gu) {
        S.rho[3 * k + c] = gu + h2 * sp_ + dt * sv_;
        if (k >= 1) {
          const double sp = gp + sp_;
          sv_ = gv + dt * sp_ + sv_;
          sp_ = sp;
        }
      };
      double pA, vA, uA, pB, vB, uB;
      fetch(N - 1, pA, vA, uA);
      fetch(N - 2, pB, vB, uB);
      int k = N - 1;
      for (; k - 1 >= 0; k -= 2) {
        double pC, vC, uC, pD, vD, uD;
        fetch(k - 2, pC, vC, uC);
        fetch(k - 3, pD, vD, uD);
        stage(k, pA, vA, uA);
        stage(k - 1, pB, vB, uB);
        pA = pC; vA = vC; uA = uC; pB = pD; vB = vD; uB = uD;
      }
      if (k >= 0) stage(k, pA, vA, uA);
    }
    __syncthreads();
    // rho_k,c = f_k,c + al_k pi_p,c + dt pi_v,c, al_k = dt^2 (N - k - 1/2);
    // pi_N minimises sum_k |rho_k|^2 (per coordinate, 2 x 2 normal equations)
    double s_af = 0.0, s_f = 0.0;
    const int c = lane % 3;
    for (int k = lane / 3; k < N && lane < 63; k += 21) {
      const double al = dt * dt * (N - k - 0.5);
      s_af += al * S.rho[3 * k + c];
      s_f += S.rho[3 * k + c];
    }
    // per-coordinate sums: lanes with the same lane % 3
    double t_af[3], t_f[3];
    for (int cc = 0; cc < 3; ++cc) {
      t_af[cc] = wave::sum((c == cc && lane < 63) ? s_af : 0.0);
      t_f[cc] = wave::sum((c == cc && lane < 63) ? s_f : 0.0);
    }
    double a11 = 0.0, a12 = 0.0;
    for (int k = 0; k < N; ++k) {
      const double al = dt * dt * (N - k - 0.5);
      a11 += al * al;
      a12 += dt * al;
    }
    const double a22 = N * dt * dt;
    const double det = a11 * a22 - a12 * a12;
    double pp[3], pv[3];
    for (int cc = 0; cc < 3; ++cc) {
      const double b1 = -t_af[cc], b2 = -dt * t_f[cc];
      pp[cc] = (a22 * b1 - a12 * b2) / det;
      pv[cc] = (a11 * b2 - a12 * b1) / det;
    }
    if (pi6) {
      for (int cc = 0; cc < 3; ++cc) { pi6[cc] = pp[cc]; pi6[3 + cc] = pv[cc]; }
    }
    __syncthreads();
    double rm = 0.0;
    for (int e = lane; e < 3 * N; e += kW) {
      const int k = e / 3, cc = e - 3 * (e / 3);
      const double al = dt * dt * (N - k - 0.5);
      const double ppc = cc == 0 ? pp[0] : (cc == 1 ? pp[1] : pp[2]);
      const double pvc = cc == 0 ? pv[0] : (cc == 1 ? pv[1] : pv[2]);
      const double v = S.rho[e] + al * ppc + dt * pvc;
      S.rho[e] = v;
      rm = fmax(rm, fabs(v));
    }
    rmax = wave::max(rm);
    __syncthreads();
  }
};

// RS: register slots per lane for the reachable rows (N m <= 64 RS)
template <int RS>
__global__ __launch_bounds__(kW) void mpc_kernel(MpcArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem_raw[];
  const int inst = blockIdx.x;
  if (inst >= A.n) return;
  const int N = A.N, m = A.m, mr = m + 4, RT = N * mr, lane = threadIdx.x;
  int ua = 0, ub = 0;
  {
    int t = lane < 45 ? lane : 0;
    while (t >= 9 - ua) { t -= 9 - ua; ++ua; }
    ub = ua + t;
  }
  MpcCtx C{A, carve_mpc(reinterpret_cast<double*>(smem_raw), N, m), mpc_param_layout(m), N, m, mr, RT, lane, A.dt,
           ua, ub};
  MpcSm& S = C.S;
  const MpcLayout& Ly = C.Ly;
  const double dt = A.dt;

  // ---- load
  for (int e = lane; e < Ly.total; e += kW) S.prm[e] = A.params[e];
  bool bad = false;
  for (int e = lane; e < 6 * (N + 1); e += kW) {
    const double v = A.ref[(int64_t)inst * 6 * (N + 1) + e];
    S.ref[e] = v;
    bad |= !isfinite(v);
  }
  for (int k = lane; k < N; k += kW) {
    const double* q = A.planes + ((int64_t)inst * N + k) * 4;
    const double nn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    bad |= !(nn > 0.0) || !isfinite(nn) || !isfinite(q[3]);
    const double in = nn > 0.0 ? 1.0 / nn : 0.0;
    S.pl[4 * k] = q[0] * in; S.pl[4 * k + 1] = q[1] * in; S.pl[4 * k + 2] = q[2] * in; S.pl[4 * k + 3] = q[3] * in;
  }
  double* x0 = S.tmp;          // start state, read with lane-dependent indices
  if (lane < 6) S.tmp[lane] = A.x0[6 * (int64_t)inst + lane];
  __syncthreads();
  for (int c = 0; c < 6; ++c) bad |= !isfinite(x0[c]);
  auto finish_nan = [&](int status, int its) {
    for (int e = lane; e < 6 * (N + 1); e += kW) A.X[(int64_t)inst * 6 * (N + 1) + e] = __builtin_nan("");
    for (int e = lane; e < 3 * N; e += kW) A.U[(int64_t)inst * 3 * N + e] = __builtin_nan("");
    if (lane == 0) {
      A.cost[inst] = __builtin_nan("");
      A.status[inst] = status;
      A.kkt[inst] = __builtin_nan("");
      if (A.iters) A.iters[inst] = its;
    }
  };
  if (__ballot(bad) != 0ull) { finish_nan(kInvalid, 0); return; }
  __syncthreads();

  // ---- start point: zero input up to x_{N-2}, then the two inputs that
  // reach r_N; then the Newton step of the LQ without rows (its optimum)
  for (int e = lane; e < 9 * (N - 2); e += kW) {
    const int k = e / 9, a = e - 9 * (e / 9);
    double v;
    if (a < 3) v = x0[a] + k * dt * x0[3 + a];
    else if (a < 6) v = x0[a];
    else v = 0.0;
    S.z[e] = v;
  }
  if (lane == 0) {
    double xa[6];
    for (int c = 0; c < 3; ++c) { xa[c] = x0[c] + (N - 2) * dt * x0[3 + c]; xa[3 + c] = x0[3 + c]; }
    // rhs = r_N - A^2 x_{N-2}
    double rr[6];
    for (int c = 0; c < 3; ++c) {
      rr[c] = S.ref[6 * N + c] - (xa[c] + 2.0 * dt * xa[3 + c]);
      rr[3 + c] = S.ref[6 * N + 3 + c] - xa[3 + c];
    }
    double uu[6];
    for (int i = 0; i < 6; ++i) {
      double v = 0.0;
      for (int c = 0; c < 6; ++c) v += S.prm[Ly.Mi + 6 * i + c] * rr[c];
      uu[i] = v;
    }
    double* z2 = S.z + 9 * (N - 2);
    double* z1 = S.z + 9 * (N - 1);
    for (int c = 0; c < 6; ++c) z2[c] = xa[c];
    for (int c = 0; c < 3; ++c) {
      z2[6 + c] = uu[c];
      z1[c] = xa[c] + dt * xa[3 + c] + 0.5 * dt * dt * uu[c];
      z1[3 + c] = xa[3 + c] + dt * uu[c];
      z1[6 + c] = uu[3 + c];
    }
  }
  for (int e = lane; e < RT; e += kW) S.X[e] = 0.0;     // no rows yet
  __syncthreads();
  C.factor();
  // g = H z + h
  for (int e = lane; e < 9 * N; e += kW) {
    const int k = e / 9, a = e - 9 * (e / 9);
    const double* H = C.Hk(k);
    double v = C.hk(k, a);
    for (int b = 0; b < 9; ++b) v += H[9 * a + b] * S.z[9 * k + b];
    S.g[e] = v;
  }
  __syncthreads();
  C.lq_solve();
  for (int e = lane; e < 9 * N; e += kW) S.z[e] += S.dz[e];
  __syncthreads();
  // slacks and multipliers; per row, in registers of the owning lane: slack
  // s, multiplier l and primal residual rp = c'z + s - d
  constexpr int NS = RS + 4;
  double rs[NS], rl[NS], rp[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) { rs[j] = 1.0; rl[j] = 1.0; rp[j] = 0.0; }
  C.template for_rows<RS, true, false>([&](int j, int r, double cz, double, double d) {
    rs[j] = fmax(d - cz, 1.0);
    S.X[r] = 1.0;
  });
  __syncthreads();

  // ---- interior-point iterations
  int it = 0;
  bool converged = false;
  double mu = 0.0, rpmax = 0.0, rdmax = 0.0, gscale = 0.0;
  for (;; ++it) {
    C.dual_residual(rdmax, gscale);             // multipliers in S.X
    double smu = 0.0, rpm = 0.0;
    C.template for_rows<RS, true, false>([&](int j, int r, double cz, double, double d) {
      const double v = cz + rs[j] - d;
      rp[j] = v;
      rpm = fmax(rpm, fabs(v));
      smu += rs[j] * rl[j];
      S.X[r] = div_nr(rl[j], rs[j]);            // barrier weight for the factorisation
    });
    __syncthreads();
    mu = wave::sum(smu) / RT;
    rpmax = wave::max(rpm);
    if (mu <= A.tol && rpmax <= 1e-10 && rdmax <= 1e-8 * (1.0 + gscale)) { converged = true; break; }
    if (it >= A.max_iters || !isfinite(mu)) break;
    if (!C.factor()) break;                     // a Quu lost definiteness: keep the current iterate
    // predictor: w = (l / s) rp - l
    C.template for_rows<RS, false, false>([&](int j, int r, double, double, double) {
      S.X[r] = div_nr(rl[j], rs[j]) * rp[j] - rl[j];
    });
    __syncthreads();
    C.build_g();
    C.lq_solve();
    // affine step: ds = -rp - c'dz, dl = -l - (l / s) ds; c'dz kept in S.X
    double amax_l = 1.0;
    C.template for_rows<RS, false, true>([&](int j, int r, double, double cd, double) {
      const double ds = -rp[j] - cd;
      const double dl = -rl[j] - div_nr(rl[j], rs[j]) * ds;
      if (ds < 0.0) amax_l = fmin(amax_l, div_nr(rs[j], -ds));
      if (dl < 0.0) amax_l = fmin(amax_l, div_nr(rl[j], -dl));
      S.X[r] = cd;
    });
    const double aa = wave::min(amax_l);
    double mua = 0.0;
    C.template for_rows<RS, false, false>([&](int j, int r, double, double, double) {
      const double ds = -rp[j] - S.X[r];
      const double dl = -rl[j] - div_nr(rl[j], rs[j]) * ds;
      mua += (rs[j] + aa * ds) * (rl[j] + aa * dl);
      S.X[r] = ds * dl;                         // affine product for the corrector
    });
    mua = wave::sum(mua) / RT;
    const double sc = (mua / mu) * (mua / mu) * (mua / mu);
    const double smu_t = sc * mu;
    // corrector: rc = s l + ds_aff dl_aff - sc mu, w = (l rp - rc) / s
    C.template for_rows<RS, false, false>([&](int j, int r, double, double, double) {
      const double rc = rs[j] * rl[j] + S.X[r] - smu_t;
      S.X[r] = div_nr(rl[j] * rp[j] - rc, rs[j]);
    });
    __syncthreads();
    C.build_g();
    C.lq_solve();
    // step: ds = -rp - c'dz, dl = (-rc - l ds) / s with rc = l rp - s w (w in S.X)
    double am = 1.0;
    C.template for_rows<RS, false, true>([&](int j, int r, double, double cd, double) {
      const double ds = -rp[j] - cd;
      const double rc = rl[j] * rp[j] - rs[j] * S.X[r];
      const double dl = div_nr(-rc - rl[j] * ds, rs[j]);
      if (ds < 0.0) am = fmin(am, div_nr(rs[j], -ds));
      if (dl < 0.0) am = fmin(am, div_nr(rl[j], -dl));
    });
    const double alpha = fmin(1.0, 0.995 * wave::min(am));
    bool nonfinite = !(alpha > 0.0) || !isfinite(alpha);
    for (int e = lane; e < 9 * N; e += kW) nonfinite |= !isfinite(S.dz[e]);
    if (__ballot(nonfinite) != 0ull) break;     // a broken direction: keep the current iterate
    C.template for_rows<RS, false, true>([&](int j, int r, double, double cd, double) {
      const double ds = -rp[j] - cd;
      const double rc = rl[j] * rp[j] - rs[j] * S.X[r];
      const double dl = div_nr(-rc - rl[j] * ds, rs[j]);
      rs[j] += alpha * ds;
      rl[j] += alpha * dl;
      S.X[r] = rl[j];
    });
    __syncthreads();
    for (int e = lane; e < 9 * N; e += kW) S.z[e] += alpha * S.dz[e];
    __syncthreads();
  }

  // ---- outputs: states (x_N from the dynamics), inputs, cost, residuals
  double cst = 0.0;
  for (int e = lane; e < 9 * N; e += kW) {
    const int k = e / 9, a = e - 9 * (e / 9);
    const double* H = C.Hk(k);
    double hz = 0.0;
    for (int b = 0; b < 9; ++b) hz += H[9 * a + b] * S.z[9 * k + b];
    cst += 0.5 * S.z[e] * hz + C.hk(k, a) * S.z[e];
    if (a < 6 && k >= 1) {
      double qr = 0.0;
      for (int b = 0; b < 6; ++b) qr += S.prm[Ly.Qm + 6 * a + b] * S.ref[6 * k + b];
      cst += S.ref[6 * k + a] * qr;
    }
  }
  const double cost = wave::sum(cst);
  double pres = 0.0, pscale = 0.0, cres = 0.0, lmax = 0.0;
  C.template for_rows<RS, true, false>([&](int j, int, double v, double, double d) {
    pres = fmax(pres, v - d);
    pscale = fmax(pscale, fmax(fabs(v), fabs(d)));
    cres = fmax(cres, rl[j] * fabs(d - v));
    lmax = fmax(lmax, rl[j]);
  });
  pres = wave::max(pres); pscale = wave::max(pscale); cres = wave::max(cres); lmax = wave::max(lmax);
  const double kkt = fmax(fmax(fmax(pres, 0.0) / (1.0 + pscale), rdmax / (1.0 + gscale)), cres / (1.0 + lmax));
  const int64_t xo = (int64_t)inst * 6 * (N + 1);
  for (int e = lane; e < 6 * N; e += kW) {
    const int k = e / 6, a = e - 6 * (e / 6);
    A.X[xo + e] = (k == 0) ? x0[a] : S.z[9 * k + a];
  }
  if (lane < 6) {
    const double* zl = S.z + 9 * (N - 1);
    const int c = lane % 3;
    const double v = lane < 3 ? zl[c] + dt * zl[3 + c] + 0.5 * dt * dt * zl[6 + c] : zl[3 + c] + dt * zl[6 + c];
    A.X[xo + 6 * N + lane] = v;
  }
  for (int e = lane; e < 3 * N; e += kW) A.U[(int64_t)inst * 3 * N + e] = S.z[9 * (e / 3) + 6 + e % 3];
  const bool solved = kkt <= 1e-6 && isfinite(cost);
  if (lane == 0) {
    A.cost[inst] = cost;
    A.kkt[inst] = kkt;
    A.status[inst] = solved ? kSolved : (converged ? kNumerical : kMaxIter);
    if (A.iters) A.iters[inst] = it;
  }
  if (solved || converged || !A.ubox_ok) return;

  // ---- infeasibility certificate for a horizon the iterations did not solve.
  // With w >= 0 on the rows (the last multipliers, scaled to max 1) and the
  // terminal costate pi, Phi(u) = sum_i w_i (c_i'z(u) - d_i) + pi'(x_N(u) - r_N)
  // is affine in the inputs u along trajectories of the dynamics from x0,
  // Phi(u) = Phi(0) + rho'u, and Phi(u) <= 0 for every feasible u.  Every
  // feasible u_k also lies in the input box of the rows that act on u alone.
  // So Phi(0) + min over the box of rho'u > 0 proves that no feasible
  // trajectory exists (FP64, with a margin for rounding).
  {
    double lm = 0.0;
    C.template for_rows<RS, false, false>([&](int j, int, double, double, double) { lm = fmax(lm, rl[j]); });
    lm = wave::max(lm);
    const double isc = (lm > 0.0 && isfinite(lm)) ? 1.0 / lm : 0.0;
    C.template for_rows<RS, false, false>([&](int j, int r, double, double, double) { S.X[r] = rl[j] * isc; });
    __syncthreads();
    double rdm = 0.0, gsc = 0.0, pi6[6];
    C.template dual_residual<false>(rdm, gsc, pi6);
    // free response: zero inputs from x0
    for (int e = lane; e < 9 * N; e += kW) {
      const int k = e / 9, a = e - 9 * (e / 9);
      S.z[e] = a < 3 ? x0[a] + k * dt * x0[3 + a] : (a < 6 ? x0[a] : 0.0);
    }
    __syncthreads();
    double phi = 0.0, pab = 0.0;
    C.template for_rows<RS, true, false>([&](int, int r, double cz, double, double d) {
      const double w = S.X[r];
      phi += w * (cz - d);
      pab += w * (fabs(cz) + fabs(d));
    });
    phi = wave::sum(phi);
    pab = wave::sum(pab);
    double tn = 0.0, tnab = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double ep = x0[c] + N * dt * x0[3 + c] - S.ref[6 * N + c], ev = x0[3 + c] - S.ref[6 * N + 3 + c];
      tn += pi6[c] * ep + pi6[3 + c] * ev;
      tnab += fabs(pi6[c] * ep) + fabs(pi6[3 + c] * ev);
    }
    double mb = 0.0, mbab = 0.0, umax = 0.0;
    for (int e = lane; e < 3 * N; e += kW) {
      const int c = e - 3 * (e / 3);
      const double lo = c == 0 ? A.ulo[0] : (c == 1 ? A.ulo[1] : A.ulo[2]);
      const double hi = c == 0 ? A.uhi[0] : (c == 1 ? A.uhi[1] : A.uhi[2]);
      const double r = S.rho[e];
      mb += r > 0.0 ? r * lo : r * hi;
      mbab += fabs(r) * fmax(fabs(lo), fabs(hi));
      umax = fmax(umax, fmax(fabs(lo), fabs(hi)));
    }
    mb = wave::sum(mb);
    mbab = wave::sum(mbab);
    umax = wave::max(umax);
    // rounding: relative 1e-9 of every magnitude that entered, including the
    // costate recursion behind rho (N stages, growth N dt)
    const double margin = 1e-9 * (pab + tnab + mbab + 3.0 * N * umax * gsc * N * (1.0 + N * dt)) + 1e-300;
    if (phi + tn + mb > margin && isfinite(phi + tn + mb)) {
      for (int e = lane; e < 6 * (N + 1); e += kW) A.X[xo + e] = __builtin_nan("");
      for (int e = lane; e < 3 * N; e += kW) A.U[(int64_t)inst * 3 * N + e] = __builtin_nan("");
      if (lane == 0) {
        A.cost[inst] = __builtin_huge_val();
        A.kkt[inst] = __builtin_nan("");
        A.status[inst] = kInfeasible;
      }
    }
  }
}

}  // namespace

size_t mpc_lds_bytes(int N, int m) { return sizeof(double) * size_t(mpc_lds_doubles(N, m)); }

hipError_t launch_mpc(const MpcArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const size_t lds = mpc_lds_bytes(a.N, a.m);
  // register slots for the reachable rows; the plane rows (4 N <= 256) take
  // four more
  const int rows = a.N * a.m;
  if (a.N < 2 || a.N > 64 || a.m < 0 || rows > 32 * kW) return hipErrorInvalidValue;
  if (rows <= 8 * kW)
    hipLaunchKernelGGL(mpc_kernel<8>, dim3(a.n), dim3(kW), lds, s, a);
  else if (rows <= 16 * kW)
    hipLaunchKernelGGL(mpc_kernel<16>, dim3(a.n), dim3(kW), lds, s, a);
  else
    hipLaunchKernelGGL(mpc_kernel<32>, dim3(a.n), dim3(kW), lds, s, a);
  return hipGetLastError();
}

}  // namespace rbp
