// Per-degree constant tables of the segment problem, built once on the host
// in FP64 and uploaded to device constant memory.
//
// A degree-p curve on [0,T] (Sec. II-B of the paper) has second-derivative
// control points p(p-1)/T^2 * Delta^2 P_k on the degree-(p-2) Bernstein basis,
// so  int_0^T |b''|^2 dt = T^-3 * sum_c P[:,c]^T Q1 P[:,c]  with
//   Q1 = (p(p-1))^2 * D2^T M D2,   M_ij = C(n,i)C(n,j) / ((2n+1) C(2n,i+j)),
// n = p-2 (the Bernstein Gram matrix).  With both end points pinned the
// interior block 2*Q1[1:p,1:p] is positive definite; its Cholesky factor L1
// whitens the objective of the reduced problem (the same factor acts on each
// coordinate because the Hessian is Q1 (x) I3).
#pragma once
#include <cmath>
#include <cstring>

namespace rbp {

constexpr int kMinDeg = 3;
constexpr int kMaxDeg = 9;
constexpr int kMaxPts = kMaxDeg + 1;      // control points
constexpr int kMaxFree = kMaxDeg - 1;     // interior (free) control points
constexpr int kMaxN = 3 * kMaxFree;       // free variables
constexpr int kMaxCol = 3 * kMaxPts;      // coefficients of one full row

struct DegConst {
  double Q1[kMaxPts][kMaxPts];        // T = 1 Hessian per coordinate
  double L1[kMaxFree][kMaxFree];      // chol(2 Q1[1:p,1:p]), lower
  double L1inv[kMaxFree][kMaxFree];   // its inverse, lower
  double kappa[kMaxFree];             // squared column norms of L1inv
  double wn_vel[kMaxDeg];             // whitened norm of velocity row k (T = 1)
  double wn_acc[kMaxDeg];             // whitened norm of acceleration row k (T = 1)
  double Gdiff[kMaxFree][kMaxFree];   // sum over vel/acc rows of a a^T / |L1inv a|^2 (T = 1)
  double rkappa[kMaxFree];            // 1 / sqrt(kappa)
  double rwn_vel[kMaxDeg];            // 1 / wn_vel
  double rwn_acc[kMaxDeg];            // 1 / wn_acc
};

inline double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Fill tables for one degree p.  Returns false if the interior block is not
// positive definite (cannot happen for 3 <= p <= 9).
inline bool build_degree(int p, DegConst& c) {
  std::memset(&c, 0, sizeof(c));
  const int np = p + 1, nf = p - 1, n2 = p - 2;
  // second-difference operator D2: (p-1) x (p+1)
  double D2[kMaxPts][kMaxPts] = {};
  for (int k = 0; k < nf; ++k) { D2[k][k] = 1.0; D2[k][k + 1] = -2.0; D2[k][k + 2] = 1.0; }
  double M[kMaxPts][kMaxPts] = {};
  for (int i = 0; i <= n2; ++i)
    for (int j = 0; j <= n2; ++j)
      M[i][j] = binom(n2, i) * binom(n2, j) / ((2.0 * n2 + 1.0) * binom(2 * n2, i + j));
  const double s = double(p) * (p - 1);
  for (int a = 0; a < np; ++a)
    for (int b = 0; b < np; ++b) {
      double acc = 0.0;
      for (int i = 0; i <= n2; ++i)
        for (int j = 0; j <= n2; ++j) acc += D2[i][a] * M[i][j] * D2[j][b];
      c.Q1[a][b] = s * s * acc;
    }
  // Cholesky of the interior block (times 2: objective written as 1/2 x^T P x)
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = 2.0 * c.Q1[i + 1][j + 1];
      for (int k = 0; k < j; ++k) v -= c.L1[i][k] * c.L1[j][k];
      if (i == j) {
        if (!(v > 0.0)) return false;
        c.L1[i][i] = std::sqrt(v);
      } else {
        c.L1[i][j] = v / c.L1[j][j];
      }
    }
  // inverse of the lower factor by forward substitution on unit vectors
  for (int col = 0; col < nf; ++col)
    for (int i = 0; i < nf; ++i) {
      double v = (i == col) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= c.L1[i][k] * c.L1inv[k][col];
      c.L1inv[i][col] = v / c.L1[i][i];
    }
  for (int k = 0; k < nf; ++k) {
    double a = 0.0;
    for (int i = 0; i < nf; ++i) a += c.L1inv[i][k] * c.L1inv[i][k];
    c.kappa[k] = a;
  }
  // difference rows restricted to interior points (1-D), T = 1 scalings
  auto whiten_norm_and_gram = [&](const double* a1, double* wn) {
    double w[kMaxFree];
    double nn = 0.0;
    for (int i = 0; i < nf; ++i) {
      double v = 0.0;
      for (int t = 0; t <= i; ++t) v += c.L1inv[i][t] * a1[t];
      w[i] = v;
      nn += v * v;
    }
    *wn = std::sqrt(nn);
    if (nn > 0.0)
      for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nf; ++j) c.Gdiff[i][j] += a1[i] * a1[j] / nn;
  };
  for (int k = 0; k < p; ++k) {            // velocity: p (P_{k+1} - P_k)
    double a1[kMaxFree] = {};
    if (k + 1 >= 1 && k + 1 <= nf) a1[k] += p;
    if (k >= 1 && k <= nf) a1[k - 1] -= p;
    whiten_norm_and_gram(a1, &c.wn_vel[k]);
    // each 1-D row appears twice (two-sided) in the ADMM constraint set but
    // with a single z; the Gram term counts it once.
  }
  for (int k = 0; k < p - 1; ++k) {        // acceleration: p(p-1) (P_{k+2} - 2P_{k+1} + P_k)
    double a1[kMaxFree] = {};
    const double sa = double(p) * (p - 1);
    if (k + 2 >= 1 && k + 2 <= nf) a1[k + 1] += sa;
    if (k + 1 >= 1 && k + 1 <= nf) a1[k] -= 2.0 * sa;
    if (k >= 1 && k <= nf) a1[k - 1] += sa;
    whiten_norm_and_gram(a1, &c.wn_acc[k]);
  }
  for (int k = 0; k < nf; ++k) c.rkappa[k] = 1.0 / std::sqrt(c.kappa[k]);
  for (int k = 0; k < p; ++k) c.rwn_vel[k] = 1.0 / c.wn_vel[k];
  for (int k = 0; k < p - 1; ++k) c.rwn_acc[k] = 1.0 / c.wn_acc[k];
  return true;
}

}  // namespace rbp
