// Multi-segment paths: S degree-p segments joined with continuous position,
// velocity and acceleration, one 64-lane wavefront per path.
//
// Each segment keeps its control points in its own free-space polytope
// (Property 1 of the paper), respects the velocity and acceleration bounds
// and its reachable Bezier polytope (Theorem 2) from its own start state
// (the path's start state for the first segment, the join state
// (P^s_0, p/T (P^s_1 - P^s_0)) for the others); start and goal are pinned.
//
// Elimination of the joins.  With equal durations, C0/C1/C2 fix the first
// three control points of segment s >= 1 from the last three of segment s-1:
//   P^s_0 = w2,  P^s_1 = 2 w2 - w1,  P^s_2 = 4 w2 - 4 w1 + w0,  P^s_k = w_k (k >= 3)
// for the window w = (P^{s-1}_{p-2}, P^{s-1}_{p-1}, P^{s-1}_p, P^s_3 .. P^s_p).
// The free variables are the "global points" g_1 .. g_{NG-2} (g_0 = start,
// g_{NG-1} = goal); segment s reads the p+1 consecutive global points from
// ws(s) = (p-2) s.  The cost is sum_c g_c^T G1 g_c with G1 banded (bandwidth
// p), so the Hessian is G1 (x) I3.
//
// Forward pass: FP32 ADMM warm start with the banded K = P + rho A^T D^2 A
// factored in LDS; FP64 dual active-set polish (Goldfarb-Idnani in the
// Hessian's metric) using banded Cholesky solves with G1 (one lane per global
// point) and a dense Cholesky factor of the small Schur complement
// N^T G^-1 N of the working set; Farkas vectors verified in FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "rbp_internal.hpp"
#include "rbp_wave.hpp"

namespace rbp {

__constant__ DegConst c_chain_deg[kMaxDeg + 1];

namespace {

constexpr int kWave = 64;
constexpr int kSolved = 0, kInfeasible = 1, kPolishFailed = 3, kNumerical = 4, kInvalid = 5;
// internal: the working set outgrew a reduced-cap pass; the full-cap pass
// that follows continues the path from the working set it stored and
// overwrites every output
constexpr int kRetry = 6;
constexpr float kBigF = 1e30f;
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ double sel3(int c, double a, double b, double d) {
  return c == 0 ? a : (c == 1 ? b : d);
}

template <int P>
struct CLds {
  static constexpr int NP = P + 1, NC = 3 * (P + 1), BW = 3 * (P + 1) - 1;
  int *nf, *nr, *f0, *rowoff;
  int64_t *r0, *hb;
  double *Af, *bfs, *rb, *Pseg, *gfull, *G1b, *L1b, *L1r, *qv, *xu, *x, *scal;
  float *fan, *rn;
  int* cand;
  unsigned* actbits;
  // ADMM region
  float *Kb, *zr, *yr, *accp, *Pf, *xt, *Cs;
  double* Wm;
  // polish region
  double *LS, *LSd, *beta, *acte, *u, *w, *zv, *np, *cvec;
  int *actid, *actside, *actseg;
};

template <int P>
__device__ CLds<P> ccarve(char* s, const ChainDims& D) {
  CLds<P> L;
  L.nf = (int*)(s + D.o_segi);
  L.nr = L.nf + D.s_cap;
  L.f0 = L.nr + D.s_cap;
  L.rowoff = L.f0 + D.s_cap;             // s_cap + 1 entries
  L.r0 = (int64_t*)(s + D.o_seg64);
  L.hb = L.r0 + D.s_cap;
  L.Af = (double*)(s + D.o_Af);
  L.bfs = (double*)(s + D.o_bfs);
  L.fan = (float*)(s + D.o_fan);
  L.rb = (double*)(s + D.o_rb);
  L.rn = (float*)(s + D.o_rn);
  L.Pseg = (double*)(s + D.o_Pseg);
  L.gfull = (double*)(s + D.o_gfull);
  L.G1b = (double*)(s + D.o_G1b);
  L.L1b = (double*)(s + D.o_L1b);
  L.L1r = (double*)(s + D.o_L1r);
  L.qv = (double*)(s + D.o_qv);
  L.xu = L.qv + 3 * D.nf_pts_cap;
  L.x = (double*)(s + D.o_x);
  L.scal = (double*)(s + D.o_scal);
  L.cand = (int*)(s + D.o_cand);
  L.actbits = (unsigned*)(s + D.o_bits);
  L.Kb = (float*)(s + D.o_Kb);
  L.zr = (float*)(s + D.o_zr);
  L.yr = (float*)(s + D.o_yr);
  L.accp = (float*)(s + D.o_accp);
  L.Pf = (float*)(s + D.o_Pf);
  L.xt = (float*)(s + D.o_xt);
  L.Cs = (float*)(s + D.o_Cs);
  L.Wm = (double*)(s + D.o_Wm);
  L.LS = (double*)(s + D.o_LS);
  L.LSd = (double*)(s + D.o_LSd);
  L.beta = (double*)(s + D.o_beta);
  L.acte = (double*)(s + D.o_acte);
  L.u = (double*)(s + D.o_u);
  L.w = L.u + D.n_cap;
  L.zv = L.w + D.n_cap;
  L.np = L.zv + D.n_cap;
  L.cvec = (double*)(s + D.o_cvec);
  L.actid = (int*)(s + D.o_actid);
  L.actside = L.actid + D.q_cap;
  L.actseg = L.actside + D.q_cap;
  return L;
}

// window map of segment s >= 1: control point k as a combination of window
// points (coefficients for w0, w1, w2; identity for k >= 3)
__device__ __forceinline__ double mcoef(int s, int k, int j) {
  if (s == 0 || k >= 3) return (k == j) ? 1.0 : 0.0;
  if (k == 0) return j == 2 ? 1.0 : 0.0;
  if (k == 1) return j == 2 ? 2.0 : (j == 1 ? -1.0 : 0.0);
  return j == 2 ? 4.0 : (j == 1 ? -4.0 : (j == 0 ? 1.0 : 0.0));   // k == 2
}

template <int P>
__device__ __forceinline__ void chain_instance(const ChainArgs& A, const int ch, char* smem) {
  using L_t = CLds<P>;
  constexpr int NP = L_t::NP, NC = L_t::NC, BW = L_t::BW;
  const int lane = threadIdx.x;
  const DegConst& K = c_chain_deg[P];
  const ChainDims& D = A.dims;
  L_t L = ccarve<P>(smem, D);

  const int64_t s0 = A.seg_off[ch];
  const int S = int(A.seg_off[ch + 1] - s0);
  const int NF = (P - 1) + (S - 1) * (P - 2);   // free global points
  const int NG = NF + 2;
  const int n = 3 * NF;
  const double T = A.T, T15 = T * sqrt(T), iT3 = 1.0 / (T * T * T);
  const double sv = double(P) / T, sa = double(P) * (P - 1) / (T * T);
  double x0[6], dg[3];
  bool bad = false;
  for (int e = 0; e < 6; ++e) { x0[e] = A.x0[6 * (int64_t)ch + e]; bad |= !isfinite(x0[e]); }
  for (int c = 0; c < 3; ++c) { dg[c] = A.goal[3 * (int64_t)ch + c] - x0[c]; bad |= !isfinite(dg[c]); }
  const int64_t pbase = (int64_t)NC * s0;   // output offset (doubles)
  (void)T15;

  auto finish = [&](int status) {
    for (int e = lane; e < S * NC; e += kWave) A.P_out[pbase + e] = __builtin_nan("");
    if (lane == 0) {
      A.cost_out[ch] = status == kInfeasible ? __builtin_huge_val() : __builtin_nan("");
      A.status_out[ch] = status;
      A.kkt_out[ch] = __builtin_nan("");
    }
  };

  // ---- segment tables
  if (lane < S) {
    const int64_t sg = s0 + lane;
    const int poly = A.poly_idx[sg];
    L.f0[lane] = A.poly_off[poly];
    L.nf[lane] = A.poly_off[poly + 1] - A.poly_off[poly];
    L.r0[lane] = A.reach_off[sg];
    L.nr[lane] = int(A.reach_off[sg + 1] - A.reach_off[sg]);
    L.hb[lane] = A.H_off[sg];
  }
  __syncthreads();
  if (lane == 0) {
    int acc = 0;
    for (int s = 0; s < S; ++s) { L.rowoff[s] = acc; acc += NP * L.nf[s] + 6 * P - 3 + L.nr[s]; }
    L.rowoff[S] = acc;
  }
  __syncthreads();
  const int m = L.rowoff[S];
  const int NFC = D.nf_cap, RC = D.r_cap;
  // faces (shifted bound) and reachable rows (shifted bound, 1/|alpha|)
  for (int s = 0; s < S; ++s) {
    const int nf = L.nf[s], nr = L.nr[s];
    for (int j = lane; j < nf; j += kWave) {
      const int64_t f = L.f0[s] + j;
      double a[3], an = 0.0;
      for (int c = 0; c < 3; ++c) { a[c] = A.A_face[3 * f + c]; L.Af[(s * NFC + j) * 3 + c] = a[c]; an += a[c] * a[c]; }
      const double b = A.b_face[f];
      L.bfs[s * NFC + j] = b - (a[0] * x0[0] + a[1] * x0[1] + a[2] * x0[2]);
      L.fan[s * NFC + j] = float(1.0 / sqrt(an));
      bad |= !(an > 0.0) || !isfinite(b);
    }
    for (int l = lane; l < nr; l += kWave) {
      const int64_t rr = L.r0[s] + l;
      const double* H = A.H + L.hb[s] + (int64_t)l * NC;
      const double* G = A.G + 6 * rr;
      double hs[3] = {0, 0, 0};
      double alpha2 = 0.0;
      for (int k = 0; k < NP; ++k)
        for (int c = 0; c < 3; ++c) hs[c] += H[3 * k + c];
      double b = A.h0[rr] - (hs[0] * x0[0] + hs[1] * x0[1] + hs[2] * x0[2]);
      if (s == 0) { for (int e = 0; e < 6; ++e) b += G[e] * x0[e]; }
      else { for (int c = 0; c < 3; ++c) b += G[c] * x0[c]; }
      for (int k = 0; k < NP; ++k)
        for (int c = 0; c < 3; ++c) {
          double a = H[3 * k + c];
          if (s > 0 && k == 0) a += -G[c] + sv * G[3 + c];
          if (s > 0 && k == 1) a += -sv * G[3 + c];
          alpha2 += a * a;
        }
      L.rb[s * RC + l] = b;
      L.rn[s * RC + l] = float(alpha2 > 0.0 ? 1.0 / sqrt(alpha2) : 0.0);
      bad |= !isfinite(b);
    }
  }
  if (__ballot(bad) != 0ull) { finish(kInvalid); return; }
  // the velocity rows chained along the joined polygon (S p edges) bound
  // every coordinate of goal - start by S vmax T: beyond that no path exists
  if (__ballot(lane < 3 && fabs(sel3(lane, dg[0], dg[1], dg[2])) > S * A.vmax * T * (1.0 + 1e-12)) != 0ull) {
    if (lane == 0 && A.iters_out) { A.iters_out[2 * ch] = 0; A.iters_out[2 * ch + 1] = 0; }
    finish(kInfeasible);
    return;
  }

  // ---- row helpers (local row numbering within segment s)
  // value of row (s, loc) on the control points of segment s (array Pp, stride 1)
  auto row_value = [&](int s, int loc, const double* Pp) -> double {
    const int nf = L.nf[s];
    const int F = NP * nf;
    if (loc < F) {
      const int k = loc / nf, j = loc - k * nf;
      const double* a = L.Af + (s * NFC + j) * 3;
      return a[0] * Pp[3 * k] + a[1] * Pp[3 * k + 1] + a[2] * Pp[3 * k + 2];
    }
    if (loc < F + 3 * P) {
      const int l = loc - F, k = l / 3, c = l - 3 * (l / 3);
      return sv * (Pp[3 * (k + 1) + c] - Pp[3 * k + c]);
    }
    if (loc < F + 6 * P - 3) {
      const int l = loc - F - 3 * P, k = l / 3, c = l - 3 * (l / 3);
      return sa * (Pp[3 * (k + 2) + c] - 2.0 * Pp[3 * (k + 1) + c] + Pp[3 * k + c]);
    }
    const int l = loc - F - 6 * P + 3;
    const double* H = A.H + L.hb[s] + (int64_t)l * NC;
    double v = 0.0;
    for (int e = 0; e < NC; ++e) v += H[e] * Pp[e];
    if (s > 0) {
      const double* G = A.G + 6 * (L.r0[s] + l);
      for (int c = 0; c < 3; ++c) v += (-G[c] + sv * G[3 + c]) * Pp[c] - sv * G[3 + c] * Pp[3 + c];
    }
    return v;
  };
  // bounds of row (s, loc): lo, hi (lo = -inf for one-sided rows)
  auto row_bounds = [&](int s, int loc, double& lo, double& hi) {
    const int nf = L.nf[s];
    const int F = NP * nf;
    if (loc < F) { lo = -__builtin_huge_val(); hi = L.bfs[s * NFC + (loc - (loc / nf) * nf)]; }
    else if (loc < F + 3 * P) { lo = -A.vmax; hi = A.vmax; }
    else if (loc < F + 6 * P - 3) { lo = -A.amax; hi = A.amax; }
    else { lo = -__builtin_huge_val(); hi = L.rb[s * RC + (loc - F - 6 * P + 3)]; }
  };
  // 1/|alpha| of a row (ADMM scaling, normalisation of violations)
  auto row_scale = [&](int s, int loc) -> double {
    const int nf = L.nf[s];
    const int F = NP * nf;
    if (loc < F) return L.fan[s * NFC + (loc - (loc / nf) * nf)];
    if (loc < F + 3 * P) return 1.0 / (sv * 1.4142135623730951);
    if (loc < F + 6 * P - 3) return 1.0 / (sa * 2.449489742783178);
    return L.rn[s * RC + (loc - F - 6 * P + 3)];
  };
  // control-point coefficient alpha_e (e = 3k + c) of row (s, loc)
  auto alpha_at = [&](int s, int loc, int e) -> double {
    const int nf = L.nf[s];
    const int F = NP * nf;
    const int ke = e / 3, ce = e - 3 * (e / 3);
    if (loc < F) {
      const int k = loc / nf, j = loc - k * nf;
      return ke == k ? L.Af[(s * NFC + j) * 3 + ce] : 0.0;
    }
    if (loc < F + 3 * P) {
      const int l = loc - F, k = l / 3, c = l - 3 * (l / 3);
      if (ce != c) return 0.0;
      return ke == k + 1 ? sv : (ke == k ? -sv : 0.0);
    }
    if (loc < F + 6 * P - 3) {
      const int l = loc - F - 3 * P, k = l / 3, c = l - 3 * (l / 3);
      if (ce != c) return 0.0;
      return ke == k + 2 ? sa : (ke == k + 1 ? -2.0 * sa : (ke == k ? sa : 0.0));
    }
    const int l = loc - F - 6 * P + 3;
    double a = A.H[L.hb[s] + (int64_t)l * NC + e];
    if (s > 0 && ke <= 1) {
      const double* G = A.G + 6 * (L.r0[s] + l);
      a += (ke == 0) ? (-G[ce] + sv * G[3 + ce]) : (-sv * G[3 + ce]);
    }
    return a;
  };
  // segment of a chain row id
  auto seg_of = [&](int id) -> int {
    int s = 0;
    while (s + 1 < S && L.rowoff[s + 1] <= id) ++s;
    return s;
  };
  // global full point vector from the free points x (n, interleaved xyz),
  // then the control points of every segment (shifted frame)
  auto build_points = [&](const double* xv) {
    for (int e = lane; e < 3 * NG; e += kWave) {
      const int g = e / 3, c = e - 3 * (e / 3);
      double v;
      if (g == 0) v = 0.0;
      else if (g == NG - 1) v = sel3(c, dg[0], dg[1], dg[2]);
      else v = xv[3 * (g - 1) + c];
      L.gfull[e] = v;
    }
    __syncthreads();
    for (int e = lane; e < S * NC; e += kWave) {
      const int s = e / NC, r = e - NC * (e / NC), k = r / 3, c = r - 3 * (r / 3);
      const int ws = (P - 2) * s;
      double v = 0.0;
      for (int j = 0; j < 3; ++j) v += mcoef(s, k, j) * L.gfull[3 * (ws + j) + c];
      if (k >= 3) v = L.gfull[3 * (ws + k) + c];
      L.Pseg[e] = v;
    }
    __syncthreads();
  };

  // ---- Hessian G1 (banded, bandwidth P) and its Cholesky factor on the free points
  // window Hessians: Wm[0] = 2 Q1 / T^3 (segment 0), Wm[1] = M^T Wm[0] M
  for (int e = lane; e < NP * NP; e += kWave) {
    const int a = e / NP, b = e - NP * (e / NP);
    L.Wm[e] = 2.0 * iT3 * K.Q1[a][b];
    double v = 0.0;
    for (int k = 0; k < NP; ++k)
      for (int k2 = 0; k2 < NP; ++k2) v += mcoef(1, k, a) * 2.0 * iT3 * K.Q1[k][k2] * mcoef(1, k2, b);
    L.Wm[NP * NP + e] = v;
  }
  __syncthreads();
  for (int e = lane; e < NG * (P + 1); e += kWave) {
    const int g = e / (P + 1), d = e - (P + 1) * (e / (P + 1));
    const int h = g - d;
    double v = 0.0;
    if (h >= 0) {
      for (int s = 0; s < S; ++s) {
        const int ws = (P - 2) * s;
        if (g >= ws && g <= ws + P && h >= ws) v += L.Wm[(s > 0 ? NP * NP : 0) + (g - ws) * NP + (h - ws)];
      }
    }
    L.G1b[e] = v;
  }
  __syncthreads();
  // band Cholesky of the free block (global points 1..NG-2 -> i = g-1), right-looking
  for (int e = lane; e < NF * (P + 1); e += kWave) {
    const int i = e / (P + 1), d = e - (P + 1) * (e / (P + 1));
    L.L1b[e] = (i - d >= 0) ? L.G1b[(i + 1) * (P + 1) + d] : 0.0;
  }
  __syncthreads();
  for (int i = 0; i < NF; ++i) {
    const double piv = L.L1b[i * (P + 1)];
    const double dd = sqrt(fmax(piv, 1e-300));
    __syncthreads();
    if (lane == 0) L.L1b[i * (P + 1)] = dd;
    if (lane >= 1 && lane <= P && i + lane < NF) L.L1b[(i + lane) * (P + 1) + lane] /= dd;
    __syncthreads();
    // trailing update of the band: (k, j) with i < j <= k <= i + P
    if (lane < P * (P + 1) / 2) {
      int a = 0, rem = lane;
      while (rem > a) { rem -= a + 1; ++a; }
      const int kk = i + 1 + a, jj = i + 1 + rem;   // jj <= kk
      if (kk < NF) {
        const double lk = L.L1b[kk * (P + 1) + (kk - i)], lj = L.L1b[jj * (P + 1) + (jj - i)];
        L.L1b[kk * (P + 1) + (kk - jj)] -= lk * lj;
      }
    }
    __syncthreads();
  }
  // banded solves with G1 (x) I3: lane = free point, 3 coordinates per lane
  // G = L L^T on the points (the same banded factor for each coordinate):
  // forward half-solve leaves y = L^-1 rhs in registers (lane = point),
  // backward half-solve writes L^-T y; reciprocal diagonal in L1r
  for (int i = lane; i < NF; i += kWave) L.L1r[i] = 1.0 / L.L1b[i * (P + 1)];
  __syncthreads();
  // Banded forward / backward solves, one lane per free point.  The band
  // coefficient a lane needs at a point and that point's reciprocal pivot do
  // not depend on the solution: they are loaded two points ahead (the loop
  // handles two points per pass), from addresses clamped into the factor, and
  // lanes outside the band multiply theirs by zero (the clamped entries are
  // finite), so no load waits behind a branch.
  auto gfwd = [&](const double* rhs, double& y0, double& y1, double& y2) {
    y0 = 0; y1 = 0; y2 = 0;
    if (lane < NF) { y0 = rhs[3 * lane]; y1 = rhs[3 * lane + 1]; y2 = rhs[3 * lane + 2]; }
    const int jj = lane < NF ? lane : NF - 1;
    auto fetch = [&](int i, double& dinv, double& l) {      // L[lane][i] below the diagonal, else 0
      const int ic = i < NF ? i : NF - 1;
      const int d = lane - i, dc = d < 0 ? 0 : (d > P ? P : d);
      dinv = L.L1r[ic];
      l = L.L1b[jj * (P + 1) + dc] * ((d > 0 && d <= P && lane < NF) ? 1.0 : 0.0);
    };
    auto step = [&](int i, double dinv, double l) {
      const double a0 = wave::bcast(y0, i) * dinv, a1 = wave::bcast(y1, i) * dinv, a2 = wave::bcast(y2, i) * dinv;
      const bool piv = lane == i;
      y0 = piv ? a0 : y0 - l * a0;
      y1 = piv ? a1 : y1 - l * a1;
      y2 = piv ? a2 : y2 - l * a2;
    };
    if (NF <= 0) return;
    double dA, lA, dB, lB;
    fetch(0, dA, lA);
    fetch(1, dB, lB);
    int i = 0;
    for (; i + 1 < NF; i += 2) {
      double dC, lC, dD, lD;
      fetch(i + 2, dC, lC);
      fetch(i + 3, dD, lD);
      step(i, dA, lA);
      step(i + 1, dB, lB);
      dA = dC; lA = lC; dB = dD; lB = lD;
    }
    if (i < NF) step(i, dA, lA);
  };
  auto gbwd = [&](double y0, double y1, double y2, double* out) {
    auto fetch = [&](int i, double& dinv, double& l) {      // L[i][lane] above i in the band, else 0
      const int ic = i < 0 ? 0 : i;
      const int d = i - lane, dc = d < 0 ? 0 : (d > P ? P : d);
      dinv = L.L1r[ic];
      l = L.L1b[ic * (P + 1) + dc] * ((d > 0 && d <= P && i >= 0) ? 1.0 : 0.0);
    };
    auto step = [&](int i, double dinv, double l) {
      const double a0 = wave::bcast(y0, i) * dinv, a1 = wave::bcast(y1, i) * dinv, a2 = wave::bcast(y2, i) * dinv;
      const bool piv = lane == i;
      y0 = piv ? a0 : y0 - l * a0;
      y1 = piv ? a1 : y1 - l * a1;
      y2 = piv ? a2 : y2 - l * a2;
    };
    if (NF > 0) {
      double dA, lA, dB, lB;
      fetch(NF - 1, dA, lA);
      fetch(NF - 2, dB, lB);
      int i = NF - 1;
      for (; i - 1 >= 0; i -= 2) {
        double dC, lC, dD, lD;
        fetch(i - 2, dC, lC);
        fetch(i - 3, dD, lD);
        step(i, dA, lA);
        step(i - 1, dB, lB);
        dA = dC; lA = lC; dB = dD; lB = lD;
      }
      if (i >= 0) step(i, dA, lA);
    }
    if (lane < NF) { out[3 * lane] = y0; out[3 * lane + 1] = y1; out[3 * lane + 2] = y2; }
    __syncthreads();
  };
  auto gsolve = [&](const double* rhs, double* out) {
    double y0, y1, y2;
    gfwd(rhs, y0, y1, y2);
    gbwd(y0, y1, y2, out);
  };
  // linear term from the pinned goal: q = G1[free, goal] * dg; unconstrained minimiser
  for (int e = lane; e < n; e += kWave) {
    const int i = e / 3, c = e - 3 * (e / 3);
    const int g = i + 1, d = (NG - 1) - g;
    L.qv[e] = (d <= P) ? L.G1b[(NG - 1) * (P + 1) + d] * sel3(c, dg[0], dg[1], dg[2]) : 0.0;
  }
  __syncthreads();
  gsolve(L.qv, L.xu);
  for (int e = lane; e < n; e += kWave) L.xu[e] = -L.xu[e];
  __syncthreads();

  // ======================================================================
  // FP32 ADMM warm start (banded K in LDS)
  // ======================================================================
  const int K_admm = A.admm_iters;
  int ncand = 0;
  if (K_admm > 0 && !A.retry_only) {
    const float rho = A.rho, alpha = A.alpha, irho = 1.0f / A.rho;
    // K = G (x) I3 + rho * sum_s embed(M_s^T C_s M_s); band storage Kb[i][d] = K[i][i-d]
    for (int e = lane; e < n * (BW + 1); e += kWave) {
      const int i = e / (BW + 1), d = e - (BW + 1) * (e / (BW + 1));
      const int j = i - d;
      float v = 0.0f;
      if (j >= 0 && (i % 3) == (j % 3)) {
        const int gi = i / 3, gj = j / 3;
        if (gi - gj <= P) v = float(L.G1b[(gi + 1) * (P + 1) + (gi - gj)]);
      }
      L.Kb[e] = v;
    }
    __syncthreads();
    for (int s = 0; s < S; ++s) {
      // C_s in control-point space: faces, difference rows, reachable rows (matrix cores)
      const int nf = L.nf[s], nr = L.nr[s];
      double gf[6];
      {
        double a0 = 0, a1 = 0, a2 = 0, w = 0;
        if (lane < nf) {
          a0 = L.Af[(s * NFC + lane) * 3]; a1 = L.Af[(s * NFC + lane) * 3 + 1]; a2 = L.Af[(s * NFC + lane) * 3 + 2];
          w = 1.0 / (a0 * a0 + a1 * a1 + a2 * a2);
        }
        gf[0] = wave::sum(w * a0 * a0); gf[1] = wave::sum(w * a0 * a1); gf[2] = wave::sum(w * a0 * a2);
        gf[3] = wave::sum(w * a1 * a1); gf[4] = wave::sum(w * a1 * a2); gf[5] = wave::sum(w * a2 * a2);
      }
      floatx16 acc;
#pragma unroll
      for (int g = 0; g < 16; ++g) acc[g] = 0.0f;
      const int col = lane & 31, half = lane >> 5;
      for (int t = 0; 2 * t < nr; ++t) {
        const int l = 2 * t + half;
        float a = 0.0f;
        if (l < nr && col < NC) {
          const double* H = A.H + L.hb[s] + (int64_t)l * NC;
          double v = H[col];
          if (s > 0) {
            const double* G = A.G + 6 * (L.r0[s] + l);
            if (col < 3) v += -G[col] + sv * G[3 + col];
            else if (col < 6) v -= sv * G[col];
          }
          a = float(v * L.rn[s * RC + l]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, a, acc, 0, 0, 0);
      }
      for (int e = lane; e < NC * NC; e += kWave) L.Cs[e] = 0.0f;
      __syncthreads();
#pragma unroll
      for (int g = 0; g < 16; ++g) {
        const int i = 8 * (g >> 2) + 4 * half + (g & 3);
        if (i < NC && col < NC) L.Cs[i * NC + col] = acc[g];
      }
      __syncthreads();
      for (int e = lane; e < NC * NC; e += kWave) {
        const int i = e / NC, j = e - NC * (e / NC);
        const int ki = i / 3, ci = i - 3 * ki, kj = j / 3, cj = j - 3 * kj;
        float v = L.Cs[e];
        if (ki == kj) {
          const int a = ci < cj ? ci : cj, b = ci < cj ? cj : ci;
          const int ix = a == 0 ? b : (a == 1 ? 2 + b : 5);
          const double g = ix == 0 ? gf[0] : ix == 1 ? gf[1] : ix == 2 ? gf[2] : ix == 3 ? gf[3] : ix == 4 ? gf[4] : gf[5];
          v += float(g);
        }
        if (ci == cj) {
          // velocity rows k: (P_{k+1} - P_k)^2 / 2 ; acceleration rows: (D2)^2 / 6
          double dv = 0.0;
          for (int k = 0; k < P; ++k) {
            const double ai = double(ki == k + 1) - double(ki == k), aj = double(kj == k + 1) - double(kj == k);
            dv += 0.5 * ai * aj;
          }
          for (int k = 0; k < P - 1; ++k) {
            const double ai = double(ki == k + 2) - 2.0 * double(ki == k + 1) + double(ki == k);
            const double aj = double(kj == k + 2) - 2.0 * double(kj == k + 1) + double(kj == k);
            dv += ai * aj / 6.0;
          }
          v += float(dv);
        }
        L.Cs[e] = v;
      }
      __syncthreads();
      // window transform M^T C M and accumulation into the band (free points only)
      constexpr int EPL = (NC * NC + kWave - 1) / kWave;
      float tv[EPL];
#pragma unroll
      for (int ti = 0; ti < EPL; ++ti) {
        const int e = lane + kWave * ti;
        tv[ti] = 0.0f;
        if (e >= NC * NC) continue;
        const int i = e / NC, j = e - NC * (e / NC);
        const int wi = i / 3, ci = i - 3 * wi, wj = j / 3, cj = j - 3 * wj;
        double v = 0.0;
        for (int k = 0; k < NP; ++k) {
          const double mi = mcoef(s, k, wi);
          if (mi == 0.0) continue;
          for (int k2 = 0; k2 < NP; ++k2) {
            const double mj = mcoef(s, k2, wj);
            if (mj == 0.0) continue;
            v += mi * double(L.Cs[(3 * k + ci) * NC + 3 * k2 + cj]) * mj;
          }
        }
        tv[ti] = float(v) * rho;
      }
      __syncthreads();
      const int ws = (P - 2) * s;
#pragma unroll
      for (int ti = 0; ti < EPL; ++ti) {
        const int e = lane + kWave * ti;
        if (e >= NC * NC) continue;
        const int i = e / NC, j = e - NC * (e / NC);
        const int gi = ws + i / 3, gj = ws + j / 3;
        if (gi >= 1 && gi <= NG - 2 && gj >= 1 && gj <= NG - 2) {
          const int vi = 3 * (gi - 1) + (i - 3 * (i / 3)), vj = 3 * (gj - 1) + (j - 3 * (j / 3));
          if (vj <= vi) L.Kb[vi * (BW + 1) + (vi - vj)] += tv[ti];
        }
      }
      __syncthreads();
    }
    // band Cholesky of K (FP32), right-looking
    for (int i = 0; i < n; ++i) {
      const float dd = sqrtf(fmaxf(L.Kb[i * (BW + 1)], 1e-30f));
      __syncthreads();
      if (lane == 0) L.Kb[i * (BW + 1)] = dd;
      if (lane >= 1 && lane <= BW && i + lane < n) L.Kb[(i + lane) * (BW + 1) + lane] /= dd;
      __syncthreads();
      for (int t = lane; t < BW * (BW + 1) / 2; t += kWave) {
        int a = 0, rem = t;
        while (rem > a) { rem -= a + 1; ++a; }
        const int kk = i + 1 + a, jj = i + 1 + rem;
        if (kk < n) L.Kb[kk * (BW + 1) + (kk - jj)] -= L.Kb[kk * (BW + 1) + (kk - i)] * L.Kb[jj * (BW + 1) + (jj - i)];
      }
      __syncthreads();
    }
    for (int e = lane; e < m; e += kWave) { L.zr[e] = 0.0f; L.yr[e] = 0.0f; }
    __syncthreads();
    for (int it = 0; it < K_admm; ++it) {
      // control-point accumulations sum_rows alpha * d (rho (z - d c) - y)
      for (int e = lane; e < S * NC; e += kWave) {
        const int s = e / NC, r = e - NC * (e / NC), k = r / 3, c = r - 3 * (r / 3);
        const int nf = L.nf[s], nr = L.nr[s], ro = L.rowoff[s], F = NP * nf;
        // rows of the last segment carry the pinned goal as a constant part
        auto vrow = [&](int loc, float d) -> float {
          float cst = 0.0f;
          if (s == S - 1)
            cst = float(alpha_at(s, loc, 3 * P) * dg[0] + alpha_at(s, loc, 3 * P + 1) * dg[1] +
                        alpha_at(s, loc, 3 * P + 2) * dg[2]);
          return d * (rho * (L.zr[ro + loc] - d * cst) - L.yr[ro + loc]);
        };
        float t = 0.0f;
        for (int j = 0; j < nf; ++j) t += float(L.Af[(s * NFC + j) * 3 + c]) * vrow(k * nf + j, L.fan[s * NFC + j]);
        const float dv = float(1.0 / (sv * 1.4142135623730951)), da = float(1.0 / (sa * 2.449489742783178));
        if (k >= 1) t += float(sv) * vrow(F + 3 * (k - 1) + c, dv);
        if (k <= P - 1) t -= float(sv) * vrow(F + 3 * k + c, dv);
        if (k >= 2) t += float(sa) * vrow(F + 3 * P + 3 * (k - 2) + c, da);
        if (k >= 1 && k - 1 <= P - 2) t -= float(2.0 * sa) * vrow(F + 3 * P + 3 * (k - 1) + c, da);
        if (k <= P - 2) t += float(sa) * vrow(F + 3 * P + 3 * k + c, da);
        for (int l = 0; l < nr; ++l) {
          const double* H = A.H + L.hb[s] + (int64_t)l * NC;
          double a = H[3 * k + c];
          if (s > 0 && k <= 1) {
            const double* G = A.G + 6 * (L.r0[s] + l);
            a += (k == 0) ? (-G[c] + sv * G[3 + c]) : (-sv * G[3 + c]);
          }
          t += float(a) * vrow(F + 6 * P - 3 + l, L.rn[s * RC + l]);
        }
        L.accp[e] = t;
      }
      __syncthreads();
      // right-hand side on the free global points (both windows touching a point)
      for (int e = lane; e < n; e += kWave) {
        const int g = e / 3 + 1, c = e - 3 * (e / 3);
        float t = -float(L.qv[e]);
        for (int s = 0; s < S; ++s) {
          const int ws = (P - 2) * s;
          const int j = g - ws;
          if (j < 0 || j > P) continue;
          for (int k = 0; k < NP; ++k) {
            const double mk = mcoef(s, k, j);
            if (mk != 0.0) t += float(mk) * L.accp[s * NC + 3 * k + c];
          }
        }
        L.xt[e] = t;
      }
      __syncthreads();
      // x~ = K^-1 rhs with the band factor (lane i%64 holds entries i, i+64, i+128, ...)
      {
        constexpr int MAXV = 4;                 // n <= 256
        float b[MAXV];
#pragma unroll
        for (int v = 0; v < MAXV; ++v) { const int i = lane + kWave * v; b[v] = i < n ? L.xt[i] : 0.0f; }
        for (int i = 0; i < n; ++i) {
          const int sl = i >> 6;
          float bi = 0.0f;
#pragma unroll
          for (int v = 0; v < MAXV; ++v) if (v == sl) bi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b[v]), i & 63));
          const float yi = bi / L.Kb[i * (BW + 1)];
#pragma unroll
          for (int v = 0; v < MAXV; ++v) {
            const int k = lane + kWave * v;
            if (k == i) b[v] = yi;
            else if (k > i && k <= i + BW && k < n) b[v] -= L.Kb[k * (BW + 1) + (k - i)] * yi;
          }
        }
        for (int i = n - 1; i >= 0; --i) {
          const int sl = i >> 6;
          float bi = 0.0f;
#pragma unroll
          for (int v = 0; v < MAXV; ++v) if (v == sl) bi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b[v]), i & 63));
          const float yi = bi / L.Kb[i * (BW + 1)];
#pragma unroll
          for (int v = 0; v < MAXV; ++v) {
            const int k = lane + kWave * v;
            if (k == i) b[v] = yi;
            else if (k < i && k >= i - BW) b[v] -= L.Kb[i * (BW + 1) + (i - k)] * yi;
          }
        }
#pragma unroll
        for (int v = 0; v < MAXV; ++v) { const int i = lane + kWave * v; if (i < n) L.xt[i] = b[v]; }
      }
      __syncthreads();
      // control points of x~ (FP32) and row update
      for (int e = lane; e < 3 * NG; e += kWave) {
        const int g = e / 3, c = e - 3 * (e / 3);
        double v = g == 0 ? 0.0 : (g == NG - 1 ? sel3(c, dg[0], dg[1], dg[2]) : double(L.xt[3 * (g - 1) + c]));
        L.gfull[e] = v;
      }
      __syncthreads();
      for (int e = lane; e < S * NC; e += kWave) {
        const int s = e / NC, r = e - NC * (e / NC), k = r / 3, c = r - 3 * (r / 3);
        const int ws = (P - 2) * s;
        double v = 0.0;
        for (int j = 0; j < 3; ++j) v += mcoef(s, k, j) * L.gfull[3 * (ws + j) + c];
        if (k >= 3) v = L.gfull[3 * (ws + k) + c];
        L.Pseg[e] = v;
      }
      __syncthreads();
      for (int s = 0; s < S; ++s) {
        const int ms = L.rowoff[s + 1] - L.rowoff[s], ro = L.rowoff[s];
        for (int loc = lane; loc < ms; loc += kWave) {
          const float d = float(row_scale(s, loc));
          double lo, hi;
          row_bounds(s, loc, lo, hi);
          const float zh = d * float(row_value(s, loc, L.Pseg + s * NC));
          const float flo = isfinite(lo) ? d * float(lo) : -kBigF, fhi = isfinite(hi) ? d * float(hi) : kBigF;
          float z = L.zr[ro + loc], y = L.yr[ro + loc];
          const float zrl = alpha * zh + (1.0f - alpha) * z;
          float zn = zrl + y * irho;
          zn = zn < flo ? flo : (zn > fhi ? fhi : zn);
          y += rho * (zrl - zn);
          L.zr[ro + loc] = zn;
          L.yr[ro + loc] = y;
        }
      }
      __syncthreads();
    }
    // proposals: most active first (|y|), at most q_cap of them
    for (int t = 0; t < D.q_cap; ++t) {
      double best = -1.0;
      int key = 0x7fffffff;
      for (int s = 0; s < S; ++s) {
        const int ms = L.rowoff[s + 1] - L.rowoff[s], ro = L.rowoff[s];
        for (int loc = lane; loc < ms; loc += kWave) {
          const float y = L.yr[ro + loc], z = L.zr[ro + loc];
          if (y == 0.0f) continue;
          const float d = float(row_scale(s, loc));
          double lo, hi;
          row_bounds(s, loc, lo, hi);
          const float flo = isfinite(lo) ? d * float(lo) : -kBigF, fhi = isfinite(hi) ? d * float(hi) : kBigF;
          int side = 0;
          if (fhi - z < y) side = 1;
          else if (z - flo < -y) side = -1;
          if (side != 0 && double(fabsf(y)) > best) { best = fabsf(y); key = 2 * (ro + loc) + (side > 0 ? 1 : 0); }
        }
      }
      wave::argmax(best, key);
      if (!(best > 0.0) || key < 0 || (key >> 1) >= m) break;
      if (lane == 0) { L.cand[t] = key; L.yr[key >> 1] = 0.0f; }
      ++ncand;
      __syncthreads();
    }
  }
  __syncthreads();

  // ======================================================================
  // FP64 dual active-set polish
  // ======================================================================
  const int QC = D.q_cap;
  for (int e = lane; e < (m + 31) / 32; e += kWave) L.actbits[e] = 0u;
  // box of every feasible point (velocity rows chained along the joined
  // polygon from both pinned ends): free coordinate e belongs to global point
  // g = e/3 + 1 at polygon position pos(g)
  auto box_of = [&](int e, double& lo, double& hi) {
    const int g = e / 3 + 1, c = e - 3 * (e / 3);
    int pos;
    if (g <= P) pos = g;
    else { const int s2 = (g - P - 1) / (P - 2) + 1; pos = s2 * P + 3 + (g - P - 1) % (P - 2); }
    const double vv = A.vmax * T / P, dgc = sel3(c, dg[0], dg[1], dg[2]);
    lo = fmax(-pos * vv, dgc - (S * P - pos) * vv);
    hi = fmin(pos * vv, dgc + (S * P - pos) * vv);
  };
  // (G1 (x) I3) v at free coordinate e (band storage of the Hessian), with
  // |G1| entries when ``absval``
  auto gmul_at = [&](const double* v, int e, bool absval) -> double {
    const int i = e / 3, c = e - 3 * (e / 3);
    double acc = 0.0;
    for (int d = -P; d <= P; ++d) {
      const int j = i + d;
      if (j < 0 || j >= NF) continue;
      const int hi_ = i > j ? i : j, lo_ = i > j ? j : i;
      const double gv = L.G1b[(hi_ + 1) * (P + 1) + (hi_ - lo_)];
      acc += (absval ? fabs(gv) : gv) * v[3 * j + c];
    }
    return acc;
  };
  // Ub bounds 1/2 (x - x_u)' G (x - x_u) (the path's cost, whose unconstrained
  // minimum is 0: the straight line at constant speed) over the feasible
  // points, by the smaller of: over the box, with centre x_c and half-widths
  // w, |x - x_u|_G <= |x_c - x_u|_G + |x - x_c|_G and d' G d <= sum_ij |G_ij|
  // |d_i| |d_j|; and S 3 amax^2 T, since the acceleration rows bound every
  // coordinate of every control point of each segment's b'' by amax.  A dual
  // value (relative to the unconstrained minimum) above Ub proves that no
  // feasible path exists.
  double Ub = 0.0;
  {
    for (int e = lane; e < n; e += kWave) {
      double lo, hi;
      box_of(e, lo, hi);
      L.zv[e] = 0.5 * (lo + hi) - L.xu[e];
      L.w[e] = fmax(0.5 * (hi - lo), 0.0);
    }
    __syncthreads();
    double cc = 0.0, ww = 0.0;
    for (int e = lane; e < n; e += kWave) {
      cc += L.zv[e] * gmul_at(L.zv, e, false);
      ww += L.w[e] * gmul_at(L.w, e, true);
    }
    cc = wave::sum(cc);
    ww = wave::sum(ww);
    const double rt = sqrt(fmax(cc, 0.0)) + sqrt(fmax(ww, 0.0));
    Ub = fmin(0.5 * rt * rt, 3.0 * S * A.amax * A.amax * T * (1.0 + 1e-12));
    __syncthreads();
  }
  for (int e = lane; e < n; e += kWave) L.x[e] = L.xu[e];
  __syncthreads();
  int q = 0, steps = 0, status = kPolishFailed;
  // Working set of up to QC - 1 <= 127 rows: lane l holds entries l and l + 64
  // of every working-set vector (multipliers, right-hand sides of the Schur
  // solves).  L_S is stored packed by rows, row k in k + 2 slots (the spare
  // slot past the diagonal takes the Givens downdate), with its reciprocal
  // diagonal in LSd.
  double lam0 = 0.0, lam1 = 0.0;   // multipliers of entries lane and lane + 64
  const int e0 = lane, e1 = lane + kWave;
  auto lso = [](int k) -> int { return (k * (k + 3)) >> 1; };
  auto pick = [&](double v0, double v1, int k) -> double {
    return wave::bcast(k < kWave ? v0 : v1, k & (kWave - 1));
  };
  const double ftol = A.feas_tol;
  const int max_steps = A.max_steps > 0 ? A.max_steps : 8 * n + 64;

  // entering normal of (id, side): beta cache slot ``slot``; also writes the
  // global normal into L.np
  auto load_normal = [&](int id, int side, int slot) {
    const int s = seg_of(id);
    const int loc = id - L.rowoff[s];
    if (lane < NC) {
      // window coefficients beta = M_s^T alpha (per coordinate)
      const int j = lane / 3, c = lane - 3 * (lane / 3);
      double v = 0.0;
      for (int k = 0; k < NP; ++k) {
        const double mk = mcoef(s, k, j);
        if (mk != 0.0) v += mk * alpha_at(s, loc, 3 * k + c);
      }
      L.beta[slot * NC + lane] = double(side) * v;
    }
    if (lane == 0) L.actseg[slot] = s;
    __syncthreads();
    for (int e = lane; e < n; e += kWave) L.np[e] = 0.0;
    __syncthreads();
    const int ws = (P - 2) * s;
    if (lane < NC) {
      const int g = ws + lane / 3;
      if (g >= 1 && g <= NG - 2) L.np[3 * (g - 1) + (lane - 3 * (lane / 3))] = L.beta[slot * NC + lane];
    }
    __syncthreads();
  };
  // dot of the window normal in slot k with a global vector
  auto ndot = [&](int k, const double* v) -> double {
    const int ws = (P - 2) * L.actseg[k];
    double acc = 0.0;
    for (int e = 0; e < NC; ++e) {
      const int g = ws + e / 3;
      if (g >= 1 && g <= NG - 2) acc += L.beta[k * NC + e] * v[3 * (g - 1) + (e - 3 * (e / 3))];
    }
    return acc;
  };
  // c = N^T u for the working set, u in L.u
  auto nt_u = [&](double& c0, double& c1) {
    c0 = e0 < q ? ndot(e0, L.u) : 0.0;
    c1 = e1 < q ? ndot(e1, L.u) : 0.0;
  };
  // forward / backward solves with L_S on the first qq entries.  The factor
  // entries a lane needs at step k and the reciprocal pivot do not depend on
  // the solution: they are loaded two steps ahead, from addresses clamped to
  // entries the factor holds (finite), and lanes that do not take part
  // multiply theirs by zero, so no load waits behind a branch.
  auto ls_forward = [&](double& v0, double& v1, int qq) {
    if (qq <= 0) return;
    const int a0 = e0 < qq ? e0 : qq - 1, a1 = e1 < qq ? e1 : qq - 1;
    auto fetch = [&](int k, double& d, double& l0, double& l1) {   // L_S[e][k] below the diagonal
      const int kc = k < qq ? k : qq - 1;
      d = L.LSd[kc];
      l0 = L.LS[lso(a0) + (kc < a0 ? kc : a0)] * ((e0 > k && e0 < qq) ? 1.0 : 0.0);
      l1 = L.LS[lso(a1) + (kc < a1 ? kc : a1)] * ((e1 > k && e1 < qq) ? 1.0 : 0.0);
    };
    auto step = [&](int k, double d, double l0, double l1) {
      const double vk = pick(v0, v1, k) * d;
      v0 = e0 == k ? vk : v0 - l0 * vk;
      v1 = e1 == k ? vk : v1 - l1 * vk;
    };
    double dA, xA, yA, dB, xB, yB;
    fetch(0, dA, xA, yA);
    fetch(1, dB, xB, yB);
    int k = 0;
    for (; k + 1 < qq; k += 2) {
      double dC, xC, yC, dD, xD, yD;
      fetch(k + 2, dC, xC, yC);
      fetch(k + 3, dD, xD, yD);
      step(k, dA, xA, yA);
      step(k + 1, dB, xB, yB);
      dA = dC; xA = xC; yA = yC; dB = dD; xB = xD; yB = yD;
    }
    if (k < qq) step(k, dA, xA, yA);
  };
  auto ls_backward = [&](double& v0, double& v1, int qq) {
    if (qq <= 0) return;
    auto fetch = [&](int k, double& d, double& l0, double& l1) {   // L_S[k][e] left of the diagonal
      const int kc = k < 0 ? 0 : k;
      d = L.LSd[kc];
      l0 = L.LS[lso(kc) + (e0 < kc ? e0 : kc)] * (e0 < k ? 1.0 : 0.0);
      l1 = L.LS[lso(kc) + (e1 < kc ? e1 : kc)] * (e1 < k ? 1.0 : 0.0);
    };
    auto step = [&](int k, double d, double l0, double l1) {
      const double vk = pick(v0, v1, k) * d;
      v0 = e0 == k ? vk : v0 - l0 * vk;
      v1 = e1 == k ? vk : v1 - l1 * vk;
    };
    double dA, xA, yA, dB, xB, yB;
    fetch(qq - 1, dA, xA, yA);
    fetch(qq - 2, dB, xB, yB);
    int k = qq - 1;
    for (; k - 1 >= 0; k -= 2) {
      double dC, xC, yC, dD, xD, yD;
      fetch(k - 2, dC, xC, yC);
      fetch(k - 3, dD, xD, yD);
      step(k, dA, xA, yA);
      step(k - 1, dB, xB, yB);
      dA = dC; xA = xC; yA = yC; dB = dD; xB = xD; yB = yD;
    }
    if (k >= 0) step(k, dA, xA, yA);
  };
  // w = N r (global), r given by entries (r0, r1)
  auto n_times = [&](double r0, double r1, double* out) {
    for (int e = lane; e < n; e += kWave) out[e] = 0.0;
    __syncthreads();
    if (e0 < q) L.cvec[e0] = r0;
    if (e1 < q) L.cvec[e1] = r1;
    __syncthreads();
    for (int k = 0; k < q; ++k) {
      const int ws = (P - 2) * L.actseg[k];
      if (lane < NC) {
        const int g = ws + lane / 3;
        if (g >= 1 && g <= NG - 2) out[3 * (g - 1) + (lane - 3 * (lane / 3))] += L.cvec[k] * L.beta[k * NC + lane];
      }
      __syncthreads();
    }
  };
  auto set_bit = [&](int id, bool on) {
    if (lane == 0) {
      if (on) L.actbits[id >> 5] |= (1u << (id & 31));
      else L.actbits[id >> 5] &= ~(1u << (id & 31));
    }
  };
  // row constant at x = 0 (only rows of the last segment touching the goal)
  auto row_const = [&](int id) -> double {
    const int s = seg_of(id);
    if (s != S - 1) return 0.0;
    const int loc = id - L.rowoff[s];
    return alpha_at(s, loc, 3 * P) * dg[0] + alpha_at(s, loc, 3 * P + 1) * dg[1] +
           alpha_at(s, loc, 3 * P + 2) * dg[2];
  };
  // full-row bound with side: side * bound
  auto row_e = [&](int id, int side) -> double {
    const int s = seg_of(id);
    double lo, hi;
    row_bounds(s, id - L.rowoff[s], lo, hi);
    return side > 0 ? hi : -lo;
  };
  // append constraint (id, side) whose normal sits in beta slot q and np;
  // u = G^-1 np must be in L.u, c = N^T u in (c0, c1); zz = np^T u - |l|^2
  auto append_factor = [&](int id, int side, double c0, double c1, double zz) {
    double l0 = c0, l1 = c1;
    ls_forward(l0, l1, q);
    const int ro = lso(q);
    if (e0 < q) L.LS[ro + e0] = l0;
    if (e1 < q) L.LS[ro + e1] = l1;
    if (lane == 0) {
      const double dq = sqrt(zz);
      L.LS[ro + q] = dq;
      L.LSd[q] = 1.0 / dq;
      L.actid[q] = id; L.actside[q] = side;
      L.acte[q] = row_e(id, side) - double(side) * row_const(id);
    }
    set_bit(id, true);
    ++q;
    __syncthreads();
  };
  // Cholesky delete of index kd (Givens on columns of the rows below)
  auto drop = [&](int kd) {
    set_bit(L.actid[kd], false);
    __syncthreads();
    // shift rows kd+1.. up by one (packed L_S, beta slots, ids): row k + 1
    // (columns 0..k+1) becomes row k, whose spare slot takes column k + 1
    for (int k = kd; k < q - 1; ++k) {
      const int rs = lso(k + 1), rd = lso(k);
      double a0 = 0.0, a1 = 0.0, bv = 0.0;
      if (e0 <= k + 1) a0 = L.LS[rs + e0];
      if (e1 <= k + 1) a1 = L.LS[rs + e1];
      if (lane < NC) bv = L.beta[(k + 1) * NC + lane];
      int id = 0, sd = 0, sg = 0;
      double ev = 0.0;
      if (lane == 0) { id = L.actid[k + 1]; sd = L.actside[k + 1]; sg = L.actseg[k + 1]; ev = L.acte[k + 1]; }
      __syncthreads();
      if (e0 <= k + 1) L.LS[rd + e0] = a0;
      if (e1 <= k + 1) L.LS[rd + e1] = a1;
      if (lane < NC) L.beta[k * NC + lane] = bv;
      if (lane == 0) { L.actid[k] = id; L.actside[k] = sd; L.actseg[k] = sg; L.acte[k] = ev; }
      __syncthreads();
    }
    {
      // entry j takes entry j + 1 (entry 64 comes from lane 0's second slot)
      const double up0 = __shfl(lam0, (lane + 1) & (kWave - 1), kWave);
      const double up1 = __shfl(lam1, (lane + 1) & (kWave - 1), kWave);
      const double first1 = wave::bcast(lam1, 0);
      const double n0 = (lane == kWave - 1) ? first1 : up0;
      if (e0 >= kd && e0 < q - 1) lam0 = n0;
      if (e1 >= kd && e1 < q - 1) lam1 = up1;
    }
    // rows kd..q-2 now have an entry one past the diagonal: rotate columns (j, j+1)
    for (int j = kd; j < q - 1; ++j) {
      const int rj = lso(j);
      const double a = L.LS[rj + j], b = L.LS[rj + j + 1];
      const double rr = hypot(a, b);
      const double cg = rr > 0.0 ? a / rr : 1.0, sg = rr > 0.0 ? b / rr : 0.0;
      const bool w0 = e0 >= j && e0 < q - 1, w1 = e1 >= j && e1 < q - 1;
      double x10 = 0, x20 = 0, x11 = 0, x21 = 0;
      if (w0) { x10 = L.LS[lso(e0) + j]; x20 = L.LS[lso(e0) + j + 1]; }
      if (w1) { x11 = L.LS[lso(e1) + j]; x21 = L.LS[lso(e1) + j + 1]; }
      __syncthreads();
      if (w0) {
        L.LS[lso(e0) + j] = cg * x10 + sg * x20;
        L.LS[lso(e0) + j + 1] = -sg * x10 + cg * x20;
      }
      if (w1) {
        L.LS[lso(e1) + j] = cg * x11 + sg * x21;
        L.LS[lso(e1) + j + 1] = -sg * x11 + cg * x21;
      }
      __syncthreads();
    }
    --q;
    if (e0 >= q) lam0 = 0.0;
    if (e1 >= q) lam1 = 0.0;
    if (e0 < q) L.LSd[e0] = 1.0 / L.LS[lso(e0) + e0];
    if (e1 < q) L.LSd[e1] = 1.0 / L.LS[lso(e1) + e1];
    __syncthreads();
  };
  // smallest of the entries < q, lowest index on ties
  auto min_entry = [&](double v0, double v1, double& mn, int& kd) {
    mn = e0 < q ? v0 : 1.0;
    kd = e0;
    if (e1 < q && v1 < mn) { mn = v1; kd = e1; }
    wave::argmin(mn, kd);
  };
  auto nplus_dot = [&](int slot, const double* v) -> double { return ndot(slot, v); };

  // the full pass continues from the working set the reduced-cap pass held
  // when it overflowed (the same rows in the same order: appending them and
  // solving for their multipliers restores its iterate)
  if (A.retry_only) {
    ncand = A.ws_meta[2 * ch];
    steps = A.ws_meta[2 * ch + 1];
    for (int t = lane; t < ncand; t += kWave) L.cand[t] = A.ws_keys[(int64_t)ch * A.ws_stride + t];
    __syncthreads();
  }
  // ---- warm start from the ADMM proposals (or the stored working set)
  for (int t = 0; t < ncand && q < QC - 1; ++t) {
    const int key = L.cand[t];
    const int id = key >> 1, side = (key & 1) ? 1 : -1;
    if ((L.actbits[id >> 5] >> (id & 31)) & 1u) continue;
    load_normal(id, side, q);
    gsolve(L.np, L.u);
    double c0, c1;
    nt_u(c0, c1);
    const double nu = nplus_dot(q, L.u);
    double l0 = c0, l1 = c1;
    ls_forward(l0, l1, q);
    const double ll = wave::sum((e0 < q ? l0 * l0 : 0.0) + (e1 < q ? l1 * l1 : 0.0));
    const double zz = nu - ll;
    if (zz > 1e-10 * nu) append_factor(id, side, c0, c1, zz);
  }
  // dual feasibility of the working set: S lam = N^T x_u - e
  for (int guard = 0; guard <= QC; ++guard) {
    if (q == 0) break;
    double r0 = e0 < q ? ndot(e0, L.xu) - L.acte[e0] : 0.0;
    double r1 = e1 < q ? ndot(e1, L.xu) - L.acte[e1] : 0.0;
    ls_forward(r0, r1, q);
    ls_backward(r0, r1, q);
    lam0 = e0 < q ? r0 : 0.0;
    lam1 = e1 < q ? r1 : 0.0;
    double mn;
    int kd;
    min_entry(lam0, lam1, mn, kd);
    if (mn >= 0.0) break;
    drop(kd);
  }
  // dual value relative to the unconstrained minimum, 1/2 |N lam|^2 in the
  // metric G^-1 at the warm start; each step adds t (s+ - t zz / 2)
  double dual = 0.0;
  if (q > 0) {
    n_times(lam0, lam1, L.w);
    {
      double f0, f1, f2;
      gfwd(L.w, f0, f1, f2);
      dual = 0.5 * wave::sum(lane < NF ? f0 * f0 + f1 * f1 + f2 * f2 : 0.0);
    }
    gsolve(L.w, L.zv);
    for (int e = lane; e < n; e += kWave) L.x[e] = L.xu[e] - L.zv[e];
    __syncthreads();
  }
  // FP64 check of the dual bound for multipliers lp >= 0 on the entering
  // row (normal in np) and max(lam, 0) on the working set: every feasible
  // x has f(x) >= min_x f(x) + rho'x - mu'e = f(x_u) + rho'x_u -
  // 1/2 rho' G^-1 rho - mu'e  (rho = sum mu_k n_k); certified when that
  // exceeds f(x_u) + Ub.  Uses L.w and L.zv as scratch.
  auto dual_bound_certified = [&](double e_free, double lp) -> bool {
    const double m0 = e0 < q ? fmax(lam0, 0.0) : 0.0, m1 = e1 < q ? fmax(lam1, 0.0) : 0.0;
    n_times(m0, m1, L.w);
    double mb = lp * e_free, mbabs = fabs(mb);
    for (int k = 0; k < q; ++k) {
      const double t = pick(m0, m1, k) * L.acte[k];
      mb += t;
      mbabs += fabs(t);
    }
    for (int e = lane; e < n; e += kWave) L.zv[e] = lp * L.np[e] + L.w[e];
    __syncthreads();
    double f0, f1, f2;
    gfwd(L.zv, f0, f1, f2);
    const double rgr = wave::sum(lane < NF ? f0 * f0 + f1 * f1 + f2 * f2 : 0.0);
    double rxu = 0.0;
    for (int e = lane; e < n; e += kWave) rxu += L.zv[e] * L.xu[e];
    rxu = wave::sum(rxu);
    const double D = rxu - 0.5 * rgr - mb;
    __syncthreads();
    return D > Ub + 1e-9 * (fabs(rxu) + 0.5 * rgr + mbabs + Ub) + 1e-12;
  };
  int bound_tries = 0;

  // ---- main loop
  bool infeasible = false;
  while (true) {
    build_points(L.x);
    double best = -1.0;
    int key = 0x7fffffff;
    auto consider = [&](int s, int loc, int id) {
      if ((L.actbits[id >> 5] >> (id & 31)) & 1u) return;
      double lo, hi;
      row_bounds(s, loc, lo, hi);
      const double v = row_value(s, loc, L.Pseg + s * NC);
      const double d = row_scale(s, loc);
      const double vu = v - hi, vl = lo - v;
      if (vu > ftol * (1.0 + fabs(hi)) && vu * d > best) { best = vu * d; key = 2 * id + 1; }
      if (isfinite(lo) && vl > ftol * (1.0 + fabs(lo)) && vl * d > best) { best = vl * d; key = 2 * id; }
    };
    // the rows held in LDS (faces, velocity, acceleration) segment by
    // segment, then the reachable rows, whose coefficients come from global
    // memory, two segments per pass: the two kinds never share a pass, and
    // two segments' reachable rows (<= 64 together) cost one global round trip
    for (int s = 0; s < S; ++s) {
      const int nl = NP * L.nf[s] + 6 * P - 3;
      for (int loc = lane; loc < nl; loc += kWave) consider(s, loc, L.rowoff[s] + loc);
    }
    for (int s = 0; s < S; s += 2) {
      const int nl0 = NP * L.nf[s] + 6 * P - 3, r0n = L.rowoff[s + 1] - L.rowoff[s] - nl0;
      int nl1 = 0, r1n = 0;
      if (s + 1 < S) { nl1 = NP * L.nf[s + 1] + 6 * P - 3; r1n = L.rowoff[s + 2] - L.rowoff[s + 1] - nl1; }
      for (int u = lane; u < r0n + r1n; u += kWave) {
        const int sp = u < r0n ? s : s + 1;
        const int loc = u < r0n ? nl0 + u : nl1 + (u - r0n);
        consider(sp, loc, L.rowoff[sp] + loc);
      }
    }
    wave::argmax(best, key);
    if (!(best > 0.0)) { status = kSolved; break; }
    if (q >= QC - 1 && QC < A.q_full) {
      for (int k = lane; k < q; k += kWave)
        A.ws_keys[(int64_t)ch * A.ws_stride + k] = 2 * L.actid[k] + (L.actside[k] > 0 ? 1 : 0);
      if (lane == 0) { A.ws_meta[2 * ch] = q; A.ws_meta[2 * ch + 1] = steps; }
      status = kRetry;
      break;
    }
    if (steps >= max_steps || key < 0 || (key >> 1) >= m || q >= QC - 1) { status = kPolishFailed; break; }
    const int id = key >> 1, side = (key & 1) ? 1 : -1;
    const int sp = seg_of(id);
    const double val = row_value(sp, id - L.rowoff[sp], L.Pseg + sp * NC);
    const double e_full = row_e(id, side);
    double splus = double(side) * val - e_full;
    const double e_free = e_full - double(side) * row_const(id);
    load_normal(id, side, q);       // slot q holds the entering normal
    double lamp = 0.0;
    bool added = false;
    while (!added) {
      ++steps;
      gsolve(L.np, L.u);                      // u = G^-1 n+
      double c0, c1;
      nt_u(c0, c1);                           // c = N^T u
      double r0 = c0, r1 = c1;                // r = S^-1 c
      ls_forward(r0, r1, q);
      ls_backward(r0, r1, q);
      if (e0 >= q) r0 = 0.0;
      if (e1 >= q) r1 = 0.0;
      n_times(r0, r1, L.w);                   // w = N r
      // d = n+ - N r; z = G^-1 d and zz = d^T G^-1 d = |L^-1 d|^2, a sum of
      // squares that is small exactly when n+ lies in the span of N
      for (int e = lane; e < n; e += kWave) L.zv[e] = L.np[e] - L.w[e];
      __syncthreads();
      double f0, f1, f2;
      gfwd(L.zv, f0, f1, f2);
      const double zz = wave::sum(lane < NF ? f0 * f0 + f1 * f1 + f2 * f2 : 0.0);
      gbwd(f0, f1, f2, L.zv);
      const double nu = nplus_dot(q, L.u);
      const double rmax = wave::max(fmax(fabs(r0), fabs(r1)));
      double t1 = __builtin_huge_val();
      int kd = e0;
      if (e0 < q && r0 > 1e-13 * rmax) t1 = lam0 / r0;
      if (e1 < q && r1 > 1e-13 * rmax && lam1 / r1 < t1) { t1 = lam1 / r1; kd = e1; }
      wave::argmin(t1, kd);
      // below this ratio the entering normal counts as dependent: the Schur
      // solve for r carries a relative error of about cond(S) * 1e-16
      const bool zfull = zz > 1e-14 * fmax(nu, 1e-300) && zz > 0.0;
      const double t2 = zfull ? splus / zz : __builtin_huge_val();
      if (!(t1 < 1e300) && !(t2 < 1e300)) {
        // Farkas vector: 1 on the entering constraint, -r_k >= 0 on the working set
        const double wk0 = e0 < q ? fmax(-r0, 0.0) : 0.0, wk1 = e1 < q ? fmax(-r1, 0.0) : 0.0;
        n_times(wk0, wk1, L.w);
        double beta_v = e_free;
        double wabs = fabs(e_free);
        for (int k = 0; k < q; ++k) {
          const double wkk = pick(wk0, wk1, k);
          beta_v += wkk * L.acte[k];
          wabs += fabs(wkk * L.acte[k]);
        }
        // rho = n+ + N w on the free variables; minimum of rho.x over the box
        double mb = 0.0;
        bool empty = false;
        for (int e = lane; e < n; e += kWave) {
          const double rr = L.np[e] + L.w[e];
          double lo, hi;
          box_of(e, lo, hi);
          empty |= lo > hi;
          mb += rr > 0.0 ? rr * lo : rr * hi;
        }
        mb = wave::sum(mb);
        const bool ok = (__ballot(empty) != 0ull) || (beta_v < mb - 1e-12 * (1.0 + wabs));
        status = ok ? kInfeasible : kPolishFailed;
        infeasible = true;
        break;
      }
      const double t = fmin(t1, t2);
      dual += t * (splus - 0.5 * t * (zfull ? zz : 0.0));
      if (zfull) {
        for (int e = lane; e < n; e += kWave) L.x[e] -= t * L.zv[e];
      }
      if (e0 < q) lam0 -= t * r0;
      if (e1 < q) lam1 -= t * r1;
      lamp += t;
      if (zfull) splus -= t * zz;
      __syncthreads();
      // the dual value passed the box bound: try the FP64 certificate
      if (bound_tries < 4 && dual > Ub * (1.0 + 1e-9) + 1e-12) {
        ++bound_tries;
        if (dual_bound_certified(e_free, lamp)) {
          status = kInfeasible;
          infeasible = true;
          break;
        }
      }
      if (t2 <= t1) {
        append_factor(id, side, c0, c1, zz);
        if (e0 == q - 1) lam0 = lamp;
        if (e1 == q - 1) lam1 = lamp;
        added = true;
      } else {
        drop(kd);
        // the entering normal moved with the shift of the cache: reload it
        load_normal(id, side, q);
        if (steps >= max_steps) break;
      }
    }
    if (infeasible || !added) { if (!infeasible) status = kPolishFailed; break; }
  }

  if (lane == 0 && A.iters_out) { A.iters_out[2 * ch] = K_admm; A.iters_out[2 * ch + 1] = steps; }
  if (status != kSolved) { finish(status); return; }

  // ---- KKT residuals, cost, write-back
  build_points(L.x);
  double pres = 0.0, pscale = 0.0;
  for (int s = 0; s < S; ++s) {
    const int ms = L.rowoff[s + 1] - L.rowoff[s];
    for (int loc = lane; loc < ms; loc += kWave) {
      double lo, hi;
      row_bounds(s, loc, lo, hi);
      const double v = row_value(s, loc, L.Pseg + s * NC);
      pres = fmax(pres, v - hi);
      pscale = fmax(pscale, fmax(fabs(v), fabs(hi)));
      if (isfinite(lo)) pres = fmax(pres, lo - v);
    }
  }
  pres = wave::max(pres);
  pscale = wave::max(pscale);
  // stationarity on the free variables: G x + q + N lam
  n_times(fmax(lam0, 0.0), fmax(lam1, 0.0), L.w);
  double st = 0.0, sg = 0.0, sn = 0.0;
  for (int e = lane; e < n; e += kWave) {
    const int i = e / 3, c = e - 3 * (e / 3);
    double gx = 0.0;
    for (int d = -P; d <= P; ++d) {
      const int j = i + d;
      if (j < 0 || j >= NF) continue;
      const int hi_ = i > j ? i : j, lo_ = i > j ? j : i;
      gx += L.G1b[(hi_ + 1) * (P + 1) + (hi_ - lo_)] * L.x[3 * j + c];
    }
    gx += L.qv[e];
    st = fmax(st, fabs(gx + L.w[e]));
    sg = fmax(sg, fabs(gx));
    sn = fmax(sn, fabs(L.w[e]));
  }
  const double dres = wave::max(st) / (1.0 + fmax(wave::max(sg), wave::max(sn)));
  double cres = 0.0, lmax = 0.0;
  for (int k = 0; k < q; ++k) {
    const double lk = fmax(pick(lam0, lam1, k), 0.0);
    const int id = L.actid[k];
    const int s = seg_of(id);
    const double v = row_value(s, id - L.rowoff[s], L.Pseg + s * NC);
    const double slack = row_e(id, L.actside[k]) - double(L.actside[k]) * v;
    cres = fmax(cres, lk * fabs(slack));
    lmax = fmax(lmax, lk);
  }
  cres /= (1.0 + lmax);
  const double kkt = fmax(fmax(fmax(pres, 0.0) / (1.0 + pscale), dres), cres);
  // cost = sum_s sum_c P~^T Q1 P~ / T^3
  double cst = 0.0;
  for (int e = lane; e < S * NC; e += kWave) {
    const int s = e / NC, r = e - NC * (e / NC), a = r / 3, c = r - 3 * (r / 3);
    double v = 0.0;
    for (int b = 0; b < NP; ++b) v += K.Q1[a][b] * L.Pseg[s * NC + 3 * b + c];
    cst += v * L.Pseg[e];
  }
  const double cost = wave::sum(cst) * iT3;
  for (int e = lane; e < S * NC; e += kWave) A.P_out[pbase + e] = L.Pseg[e] + sel3(e % 3, x0[0], x0[1], x0[2]);
  if (lane == 0) {
    const bool ok = kkt <= A.kkt_tol && isfinite(kkt) && isfinite(cost);
    A.cost_out[ch] = cost;
    A.status_out[ch] = ok ? kSolved : kNumerical;
    A.kkt_out[ch] = kkt;
  }
}

template <int P>
__global__ __launch_bounds__(64) void chain_kernel(ChainArgs A) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int b = blockIdx.x + A.inst_base;
  if (b >= A.N) return;
  const int ch = A.order ? A.order[b] : b;
  if (A.retry_only && A.status_out[ch] != kRetry) return;
  chain_instance<P>(A, ch, smem);
}

}  // namespace

ChainDims make_chain_dims(int p, int s_cap, int nf_cap, int r_cap, int q_cap, bool admm) {
  ChainDims d{};
  d.s_cap = s_cap < 1 ? 1 : s_cap;
  d.nf_cap = nf_cap < 1 ? 1 : nf_cap;
  d.r_cap = r_cap < 1 ? 1 : r_cap;
  d.q_cap = q_cap;
  d.nf_pts_cap = (p - 1) + (d.s_cap - 1) * (p - 2);
  d.ng_cap = d.nf_pts_cap + 2;
  d.n_cap = 3 * d.nf_pts_cap;
  d.m_cap = d.s_cap * ((p + 1) * d.nf_cap + 6 * p - 3 + d.r_cap);
  const int NP = p + 1, NC = 3 * NP, BW = NC - 1;
  int o = 0;
  auto take = [&](int bytes) { const int at = o; o += (bytes + 15) & ~15; return at; };
  d.o_segi = take((4 * d.s_cap + 1) * 4);
  d.o_seg64 = take(2 * d.s_cap * 8);
  d.o_Af = take(d.s_cap * d.nf_cap * 3 * 8);
  d.o_bfs = take(d.s_cap * d.nf_cap * 8);
  d.o_fan = take(d.s_cap * d.nf_cap * 4);
  d.o_rb = take(d.s_cap * d.r_cap * 8);
  d.o_rn = take(d.s_cap * d.r_cap * 4);
  d.o_Pseg = take(d.s_cap * NC * 8);
  d.o_gfull = take(3 * d.ng_cap * 8);
  d.o_G1b = take(d.ng_cap * NP * 8);
  d.o_L1b = take(d.nf_pts_cap * NP * 8);
  d.o_L1r = take(d.nf_pts_cap * 8);
  d.o_qv = take(2 * 3 * d.nf_pts_cap * 8);
  d.o_x = take(d.n_cap * 8);
  d.o_scal = take(16 * 8);
  d.o_cand = take(d.q_cap * 4);
  d.o_bits = take(((d.m_cap + 31) / 32) * 4);
  const int region = o;
  int a = region;
  auto take_a = [&](int bytes) { const int at = a; a += (bytes + 15) & ~15; return at; };
  // the window Hessians are built during set-up whether or not ADMM runs
  d.o_Wm = take_a(2 * NP * NP * 8);
  const int setup_end = a;
  d.o_Kb = take_a(d.n_cap * (BW + 1) * 4);
  d.o_zr = take_a(d.m_cap * 4);
  d.o_yr = take_a(d.m_cap * 4);
  d.o_accp = take_a(d.s_cap * NC * 4);
  d.o_Pf = take_a(d.s_cap * NC * 4);
  d.o_xt = take_a(d.n_cap * 4);
  d.o_Cs = take_a(NC * NC * 4);
  int b = region;
  auto take_b = [&](int bytes) { const int at = b; b += (bytes + 15) & ~15; return at; };
  d.o_LS = take_b(((d.q_cap * (d.q_cap + 3)) >> 1) * 8);   // packed rows, k + 2 slots each
  d.o_LSd = take_b(d.q_cap * 8);
  d.o_beta = take_b(d.q_cap * NC * 8);
  d.o_acte = take_b(d.q_cap * 8);
  d.o_u = take_b(4 * d.n_cap * 8);
  d.o_cvec = take_b(d.q_cap * 8);
  d.o_actid = take_b(3 * d.q_cap * 4);
  // polish only: nothing of the ADMM part but the window Hessians is used
  if (!admm) a = setup_end;
  d.bytes = a > b ? a : b;
  return d;
}

hipError_t upload_chain_constants(int device) {
  (void)device;
  DegConst host[kMaxDeg + 1];
  std::memset(host, 0, sizeof(host));
  for (int p = kMinDeg; p <= kMaxDeg; ++p)
    if (!build_degree(p, host[p])) return hipErrorInvalidValue;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_chain_deg), host, sizeof(host), 0, hipMemcpyHostToDevice);
}

hipError_t launch_chains(const ChainArgs& a, hipStream_t s) {
  if (a.N - a.inst_base <= 0) return hipSuccess;
  if (a.P != 7) return hipErrorInvalidValue;
  hipLaunchKernelGGL((chain_kernel<7>), dim3(a.N - a.inst_base), dim3(kWave), a.dims.bytes, s, a);
  return hipGetLastError();
}

}  // namespace rbp
