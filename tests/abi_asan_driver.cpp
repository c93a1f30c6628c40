// Host-side check of the C ABI's argument validation under AddressSanitizer
// (the host code of the library is compiled with -fsanitize=address for this
// program; device code is not instrumented).  Every documented error path of
// the entry points is driven with malformed descriptions and options, and a
// small valid batch, cut, graph and MPC problem are run end to end, so that
// any out-of-bounds host access in the validation and set-up code aborts the
// program.  Prints one line per check; exit status 0 when every check holds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../include/rbp.h"

namespace {

int g_fail = 0;

void expect(const char* what, int rc, int want) {
  const bool ok = rc == want;
  std::printf("%s %s: rc %d (want %d)\n", ok ? "ok  " : "FAIL", what, rc, want);
  if (!ok) ++g_fail;
}

template <typename T>
T* dev(const std::vector<T>& h) {
  T* p = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&p), (h.empty() ? 1 : h.size()) * sizeof(T)) != hipSuccess) return nullptr;
  if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return p;
}

template <typename T>
std::vector<T> host(const T* d, size_t n) {
  std::vector<T> h(n);
  if (hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) h.clear();
  return h;
}

// three segments (degrees 3, 5, 7) in the box |x_c| <= 5 with two slack
// reachable rows each, from rest at the origin to a nearby goal
struct Segments {
  std::vector<int32_t> degree{3, 5, 7}, poly_off{0, 6}, poly_idx{0, 0, 0};
  std::vector<double> T{1.0, 1.0, 1.0}, A_face, b_face, H, h0, G, x0, goal;
  std::vector<int64_t> reach_off{0, 2, 4, 6}, H_off{0};
  Segments() {
    for (int c = 0; c < 3; ++c)
      for (int s = -1; s <= 1; s += 2) {
        for (int k = 0; k < 3; ++k) A_face.push_back(k == c ? double(s) : 0.0);
        b_face.push_back(5.0);
      }
    for (int i = 0; i < 3; ++i) {
      const int p = degree[size_t(i)], nc = 3 * (p + 1);
      for (int row = 0; row < 2; ++row)
        for (int e = 0; e < nc; ++e) H.push_back(e == 3 * p + row ? 1.0 : 0.0);
      H_off.push_back(H_off.back() + 2 * nc);
      for (int row = 0; row < 2; ++row) {
        h0.push_back(100.0);
        for (int k = 0; k < 6; ++k) G.push_back(0.0);
      }
      for (int k = 0; k < 6; ++k) x0.push_back(0.0);
      goal.push_back(1.0); goal.push_back(0.5); goal.push_back(-0.2);
    }
  }
};

struct DevSegments {
  int32_t *degree, *poly_off, *poly_idx;
  double *T, *A_face, *b_face, *H, *h0, *G, *x0, *goal;
  int64_t *reach_off, *H_off;
  explicit DevSegments(const Segments& s)
      : degree(dev(s.degree)), poly_off(dev(s.poly_off)), poly_idx(dev(s.poly_idx)), T(dev(s.T)),
        A_face(dev(s.A_face)), b_face(dev(s.b_face)), H(dev(s.H)), h0(dev(s.h0)), G(dev(s.G)), x0(dev(s.x0)),
        goal(dev(s.goal)), reach_off(dev(s.reach_off)), H_off(dev(s.H_off)) {}
  rbp_problem_desc desc() const {
    rbp_problem_desc d;
    std::memset(&d, 0, sizeof(d));
    d.n_instances = 3; d.n_poly = 1; d.degree = degree; d.T = T; d.poly_off = poly_off; d.A_face = A_face;
    d.b_face = b_face; d.poly_idx = poly_idx; d.reach_off = reach_off; d.H_off = H_off; d.H = H; d.h0 = h0;
    d.G = G; d.vmax = 3.0; d.amax = 5.0;
    return d;
  }
};

void segment_checks() {
  Segments s;
  DevSegments ds(s);
  const rbp_problem_desc good = ds.desc();
  rbp_batch* b = nullptr;
  expect("build: null description", rbp_build_batch(nullptr, nullptr, &b), RBP_E_INVALID);
  rbp_problem_desc d = good;
  d.vmax = 0.0;
  expect("build: vmax 0", rbp_build_batch(&d, nullptr, &b), RBP_E_INVALID);
  d = good; d.pin_start_velocity = 2;
  expect("build: pin flag 2", rbp_build_batch(&d, nullptr, &b), RBP_E_INVALID);
  d = good; d.degree = nullptr;
  expect("build: null degree", rbp_build_batch(&d, nullptr, &b), RBP_E_INVALID);
  {
    std::vector<int32_t> bad{3, 10, 7};
    int32_t* p = dev(bad);
    d = good; d.degree = p;
    expect("build: degree 10", rbp_build_batch(&d, nullptr, &b), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  {
    std::vector<int32_t> bad{1, 6};
    int32_t* p = dev(bad);
    d = good; d.poly_off = p;
    expect("build: poly_off[0] != 0", rbp_build_batch(&d, nullptr, &b), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  {
    std::vector<int32_t> bad{0, 1, 0};
    int32_t* p = dev(bad);
    d = good; d.poly_idx = p;
    expect("build: polytope index out of range", rbp_build_batch(&d, nullptr, &b), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  {
    std::vector<int64_t> bad = s.H_off;
    bad[2] += 1;
    int64_t* p = dev(bad);
    d = good; d.H_off = p;
    expect("build: H_off inconsistent with the degree", rbp_build_batch(&d, nullptr, &b), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  {
    std::vector<int64_t> bad{0, 129, 131, 133};
    int64_t* p = dev(bad);
    d = good; d.reach_off = p;
    expect("build: 129 reachable rows", rbp_build_batch(&d, nullptr, &b), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  expect("build: valid batch", rbp_build_batch(&good, nullptr, &b), RBP_OK);
  if (!b) { ++g_fail; return; }
  rbp_batch_sizes sz;
  expect("sizes", rbp_batch_get_sizes(b, &sz), RBP_OK);
  expect("sizes: null output", rbp_batch_get_sizes(b, nullptr), RBP_E_INVALID);
  const int64_t npts = sz.points_total;
  double *P = nullptr, *cost = nullptr, *kkt = nullptr, *gx = nullptr, *gg = nullptr, *gb = nullptr;
  int32_t *st = nullptr, *it = nullptr, *fl = nullptr;
  (void)hipMalloc(reinterpret_cast<void**>(&P), size_t(3 * npts) * sizeof(double));
  (void)hipMalloc(reinterpret_cast<void**>(&cost), 3 * sizeof(double));
  (void)hipMalloc(reinterpret_cast<void**>(&kkt), 3 * sizeof(double));
  (void)hipMalloc(reinterpret_cast<void**>(&st), 3 * sizeof(int32_t));
  (void)hipMalloc(reinterpret_cast<void**>(&it), 6 * sizeof(int32_t));
  (void)hipMalloc(reinterpret_cast<void**>(&gx), 18 * sizeof(double));
  (void)hipMalloc(reinterpret_cast<void**>(&gg), 9 * sizeof(double));
  (void)hipMalloc(reinterpret_cast<void**>(&gb), size_t(sz.faces_total) * sizeof(double));
  (void)hipMalloc(reinterpret_cast<void**>(&fl), 3 * sizeof(int32_t));
  expect("backward before a forward pass", rbp_backward(b, nullptr, nullptr, gx, gg, gb, fl, nullptr), RBP_E_STATE);
  rbp_solve_opts o;
  rbp_default_opts(&o);
  struct { const char* what; void (*set)(rbp_solve_opts&); } bad_opts[] = {
      {"solve: admm_iters -1", [](rbp_solve_opts& x) { x.admm_iters = -1; }},
      {"solve: rho 0", [](rbp_solve_opts& x) { x.rho = 0.0f; }},
      {"solve: launch_shape 3", [](rbp_solve_opts& x) { x.launch_shape = 3; }},
      {"solve: schedule 2", [](rbp_solve_opts& x) { x.schedule = 2; }},
      {"solve: debug_fill_lds 2", [](rbp_solve_opts& x) { x.debug_fill_lds = 2; }},
      {"solve: reserved 1", [](rbp_solve_opts& x) { x.reserved = 1; }},
  };
  for (auto& c : bad_opts) {
    rbp_solve_opts x = o;
    c.set(x);
    expect(c.what, rbp_solve_batch(b, ds.x0, ds.goal, nullptr, &x, P, cost, st, kkt, it, nullptr), RBP_E_INVALID);
  }
  expect("solve: null x0", rbp_solve_batch(b, nullptr, ds.goal, nullptr, &o, P, cost, st, kkt, it, nullptr),
         RBP_E_INVALID);
  for (int admm : {10, 0}) {
    for (int sched : {0, 1}) {
      rbp_solve_opts x = o;
      x.admm_iters = admm;
      x.schedule = sched;
      x.debug_fill_lds = 1;
      char what[96];
      std::snprintf(what, sizeof(what), "solve: valid batch (admm %d, schedule %d)", admm, sched);
      expect(what, rbp_solve_batch(b, ds.x0, ds.goal, nullptr, &x, P, cost, st, kkt, it, nullptr), RBP_OK);
      const std::vector<int32_t> hs = host(st, 3);
      const std::vector<double> hc = host(cost, 3);
      for (int i = 0; i < 3; ++i) {
        std::snprintf(what, sizeof(what), "  instance %d solved with a finite cost", i);
        expect(what, (hs.size() == 3 && hs[size_t(i)] == RBP_SOLVED && std::isfinite(hc[size_t(i)])) ? 0 : 1, 0);
      }
      expect("backward", rbp_backward(b, nullptr, nullptr, gx, gg, gb, fl, nullptr), RBP_OK);
    }
  }
  expect("backward: null grad_x0", rbp_backward(b, nullptr, nullptr, nullptr, gg, gb, fl, nullptr), RBP_E_INVALID);
  rbp_destroy_batch(b);
  rbp_destroy_batch(nullptr);
  for (void* p : {static_cast<void*>(P), static_cast<void*>(cost), static_cast<void*>(kkt), static_cast<void*>(st),
                  static_cast<void*>(it), static_cast<void*>(gx), static_cast<void*>(gg), static_cast<void*>(gb),
                  static_cast<void*>(fl)})
    (void)hipFree(p);
  for (void* p : {static_cast<void*>(ds.degree), static_cast<void*>(ds.poly_off), static_cast<void*>(ds.poly_idx),
                  static_cast<void*>(ds.T), static_cast<void*>(ds.A_face), static_cast<void*>(ds.b_face),
                  static_cast<void*>(ds.H), static_cast<void*>(ds.h0), static_cast<void*>(ds.G),
                  static_cast<void*>(ds.x0), static_cast<void*>(ds.goal), static_cast<void*>(ds.reach_off),
                  static_cast<void*>(ds.H_off)})
    (void)hipFree(p);
}

void cut_checks() {
  // two degree-3 edges, one box and one polytope (a cube written as 6 rows)
  std::vector<double> lo{2, 2, 2}, hi{3, 3, 3}, A, bb, P;
  for (int c = 0; c < 3; ++c)
    for (int s = -1; s <= 1; s += 2) {
      for (int k = 0; k < 3; ++k) A.push_back(k == c ? double(s) : 0.0);
      bb.push_back(s > 0 ? 6.0 : -5.0);
    }
  for (int e = 0; e < 2; ++e)
    for (int k = 0; k < 4; ++k) { P.push_back(k * 1.0 + e); P.push_back(0.5 * k); P.push_back(0.0); }
  std::vector<int32_t> off{0, 6};
  double *dlo = dev(lo), *dhi = dev(hi), *dA = dev(A), *db = dev(bb), *dP = dev(P);
  int32_t* doff = dev(off);
  rbp_cut_desc d;
  std::memset(&d, 0, sizeof(d));
  d.n_edges = 2; d.n_obstacles = 1; d.degree = 3; d.box_lo = dlo; d.box_hi = dhi;
  d.n_polytopes = 1; d.pob_off = doff; d.pob_A = dA; d.pob_b = db;
  rbp_cut* c = nullptr;
  expect("cut: null description", rbp_build_cut(nullptr, nullptr, &c), RBP_E_INVALID);
  rbp_cut_desc x = d;
  x.reserved = 1;
  expect("cut: reserved 1", rbp_build_cut(&x, nullptr, &c), RBP_E_INVALID);
  x = d; x.degree = 0;
  expect("cut: degree 0", rbp_build_cut(&x, nullptr, &c), RBP_E_SHAPE);
  {
    std::vector<double> ub(bb);
    ub[0] = -10.0;   // x <= -10 and x >= 5: empty
    double* p = dev(ub);
    x = d; x.pob_b = p;
    expect("cut: empty polytope", rbp_build_cut(&x, nullptr, &c), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  {
    std::vector<int32_t> o4{0, 4};   // four rows of a cube: unbounded
    int32_t* p = dev(o4);
    x = d; x.pob_off = p;
    expect("cut: unbounded polytope", rbp_build_cut(&x, nullptr, &c), RBP_E_SHAPE);
    (void)hipFree(p);
  }
  expect("cut: valid", rbp_build_cut(&d, nullptr, &c), RBP_OK);
  if (c) {
    uint8_t *code = nullptr, *step = nullptr;
    double* dist = nullptr;
    int32_t* ncol = nullptr;
    (void)hipMalloc(reinterpret_cast<void**>(&code), 4);
    (void)hipMalloc(reinterpret_cast<void**>(&step), 4);
    (void)hipMalloc(reinterpret_cast<void**>(&dist), 4 * sizeof(double));
    (void)hipMalloc(reinterpret_cast<void**>(&ncol), 2 * sizeof(int32_t));
    expect("cut: run", rbp_cut_run(c, dP, code, step, dist, ncol, nullptr), RBP_OK);
    int64_t nq = -1;
    expect("cut: undecided-pair count", rbp_cut_qp_count(c, &nq), RBP_OK);
    rbp_destroy_cut(c);
    for (void* p : {static_cast<void*>(code), static_cast<void*>(step), static_cast<void*>(dist),
                    static_cast<void*>(ncol)})
      (void)hipFree(p);
  }
  for (void* p : {static_cast<void*>(dlo), static_cast<void*>(dhi), static_cast<void*>(dA), static_cast<void*>(db),
                  static_cast<void*>(dP), static_cast<void*>(doff)})
    (void)hipFree(p);
}

void graph_checks() {
  const int n = 40, dim = 3, m = 6;
  std::vector<double> F1, F2, G, V;
  for (int k = 0; k < m; ++k) {
    for (int c = 0; c < dim; ++c) {
      const double a = (k / 2 == c) ? (k % 2 ? -1.0 : 1.0) : 0.0;
      F1.push_back(-a);
      F2.push_back(a);
    }
    G.push_back(1.5);
  }
  for (int i = 0; i < n * dim; ++i) V.push_back(0.37 * ((i * 7919) % 23));
  double *dF1 = dev(F1), *dF2 = dev(F2), *dG = dev(G), *dV = dev(V);
  rbp_graph_desc d;
  std::memset(&d, 0, sizeof(d));
  d.n_nodes = n; d.dim = dim; d.n_rows = m; d.F1 = dF1; d.F2 = dF2; d.G = dG;
  rbp_graph* g = nullptr;
  rbp_graph_desc x = d;
  x.reserved = 1;
  expect("graph: reserved 1", rbp_build_graph(&x, nullptr, &g), RBP_E_INVALID);
  x = d; x.n_rows = 0;
  expect("graph: no rows", rbp_build_graph(&x, nullptr, &g), RBP_E_SHAPE);
  expect("graph: valid", rbp_build_graph(&d, nullptr, &g), RBP_OK);
  const int words = (n + 31) / 32;
  uint32_t* adj = nullptr;
  int32_t* deg = nullptr;
  (void)hipMalloc(reinterpret_cast<void**>(&adj), size_t(n) * words * sizeof(uint32_t));
  (void)hipMalloc(reinterpret_cast<void**>(&deg), size_t(n) * sizeof(int32_t));
  if (g) {
    expect("graph: run", rbp_graph_run(g, dV, adj, deg, nullptr), RBP_OK);
    rbp_destroy_graph(g);
  }
  expect("graph without allocation: run", rbp_graph_run_noalloc(&d, dV, adj, deg, nullptr), RBP_OK);
  x = d; x.n_nodes = 20000; x.n_rows = 64;
  expect("graph without allocation: oversized", rbp_graph_run_noalloc(&x, dV, adj, deg, nullptr), RBP_E_SCRATCH);
  for (void* p : {static_cast<void*>(dF1), static_cast<void*>(dF2), static_cast<void*>(dG), static_cast<void*>(dV),
                  static_cast<void*>(adj), static_cast<void*>(deg)})
    (void)hipFree(p);
}

void mpc_checks() {
  rbp_mpc_desc d;
  std::memset(&d, 0, sizeof(d));
  d.n_instances = 1; d.horizon = 10; d.n_reach = 0; d.dt = 0.1;
  for (int i = 0; i < 6; ++i) d.Q[7 * i] = 1.0;
  for (int i = 0; i < 3; ++i) d.R[4 * i] = 0.01;
  rbp_mpc* q = nullptr;
  rbp_mpc_desc x = d;
  x.dt = 0.0;
  expect("mpc: dt 0", rbp_build_mpc(&x, nullptr, &q), RBP_E_INVALID);
  x = d; x.reserved = 1;
  expect("mpc: reserved 1", rbp_build_mpc(&x, nullptr, &q), RBP_E_INVALID);
  x = d; x.horizon = 1;
  expect("mpc: horizon 1", rbp_build_mpc(&x, nullptr, &q), RBP_E_SHAPE);
  x = d; x.R[0] = -1.0;
  expect("mpc: R not positive definite", rbp_build_mpc(&x, nullptr, &q), RBP_E_INVALID);
  expect("mpc: valid", rbp_build_mpc(&d, nullptr, &q), RBP_OK);
  if (q) rbp_destroy_mpc(q);
}

}  // namespace

int main() {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    std::printf("no GPU\n");
    return 2;
  }
  for (int code = RBP_E_SCRATCH; code <= RBP_INVALID_INPUT; ++code)
    expect("status string", rbp_status_string(code) != nullptr ? 0 : 1, 0);
  segment_checks();
  cut_checks();
  graph_checks();
  mpc_checks();
  std::printf("%s: %d failed\n", g_fail ? "FAILED" : "PASSED", g_fail);
  return g_fail ? 1 : 0;
}
