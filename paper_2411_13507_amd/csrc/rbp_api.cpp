// C ABI of the batched segment-QP library (see include/rbp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <limits>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/rbp.h"
#include "rbp_internal.hpp"

struct rbp_batch {
  int device = 0;
  rbp_problem_desc desc{};
  int32_t N = 0, pmax = 3, rmax = 0, nfmax = 1;
  // work order grouped by (degree, reachable-row class); each group is one
  // launch whose LDS is sized by the group's own largest instance
  struct Group { int32_t p, start, count, rmax, nfmax; };
  std::vector<Group> groups;
  // groups of a grouped launch run on kLanes streams at once (the caller's
  // and the device's kLanes - 1 side streams, forked from and joined back
  // into the caller's with events), assigned longest estimated cost first
  // to the least loaded stream, so that no group waits for the tail of
  // another
  static constexpr int kLanes = 4;
  std::vector<int32_t> group_lane;
  std::vector<int32_t> launch_order;   // groups by estimated cost, longest first
  hipStream_t side[kLanes - 1] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kLanes - 1] = {};
  std::vector<int32_t> degree_host;
  int64_t pt_total = 0, face_total = 0;
  int64_t* d_pt_off = nullptr;
  int64_t* d_face_off = nullptr;
  int32_t* d_order = nullptr;
  rbp::InstDesc* d_desc = nullptr;     // descriptors in work-order position
  std::vector<int32_t> pos_host;       // work-order position of each instance
  // forward state kept for backward
  int32_t nmax = 0;
  int32_t* st_q = nullptr;
  int32_t* st_id = nullptr;
  int32_t* st_side = nullptr;
  double* st_lam = nullptr;
  double* st_qr = nullptr;      // factor of the final working set (Q1 rows, R rows)
  int32_t* fw_status = nullptr;  // forward results kept for backward (written by the solve kernels)
  double* fw_nu = nullptr;      // multipliers of the pinned start and goal coordinates
  int64_t F_total = 0;
  bool has_forward = false;
  int32_t fw_schedule = 0;      // schedule of the stored forward pass
  int32_t fw_debug_fill = 0;    // its LDS NaN fill (the backward pass follows it)
  hipStream_t last_stream = nullptr;
};

namespace {
// LDS of one workgroup on gfx950
constexpr size_t kLdsBytes = 160 * 1024;

// The side streams of grouped launches: three per device, created once (at
// the first batch built on it) and shared by every batch and path batch
// of the process until it ends.  A device has few hardware queues (four by
// default), and streams beyond that share them round-robin in creation
// order: streams made per batch, after the caller's own, could land on the
// caller's queue, and groups meant to run side by side would then run one
// after another.  Made once and early, the three take consecutive queues.
std::mutex g_side_mu;
std::vector<std::pair<int, std::array<hipStream_t, 3>>> g_side;
bool side_streams(int device, hipStream_t (&out)[3]) {
  std::lock_guard<std::mutex> lk(g_side_mu);
  for (const auto& e : g_side)
    if (e.first == device) { for (int k = 0; k < 3; ++k) out[k] = e.second[k]; return true; }
  std::array<hipStream_t, 3> st{};
  for (int k = 0; k < 3; ++k)
    if (hipStreamCreateWithFlags(&st[size_t(k)], hipStreamNonBlocking) != hipSuccess) {
      for (int j = 0; j < k; ++j) (void)hipStreamDestroy(st[size_t(j)]);
      return false;
    }
  g_side.emplace_back(device, st);
  for (int k = 0; k < 3; ++k) out[k] = st[size_t(k)];
  return true;
}

std::mutex g_const_mu;
std::vector<int> g_const_done;

int ensure_constants(int device) {
  std::lock_guard<std::mutex> lk(g_const_mu);
  if (std::find(g_const_done.begin(), g_const_done.end(), device) != g_const_done.end()) return RBP_OK;
  if (rbp::upload_constants(device) != hipSuccess || rbp::upload_constants_var(device) != hipSuccess)
    return RBP_E_DEVICE;
  g_const_done.push_back(device);
  return RBP_OK;
}

template <typename T>
int dalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), n * sizeof(T)) != hipSuccess) { *p = nullptr; return RBP_E_ALLOC; }
  return RBP_OK;
}

void free_batch(rbp_batch* b) {
  if (!b) return;
  for (int k = 0; k < rbp_batch::kLanes - 1; ++k) {
    if (b->side[k]) (void)hipStreamSynchronize(b->side[k]);   // shared: not destroyed
    if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  void* ptrs[] = {b->d_pt_off, b->d_face_off, b->d_order, b->d_desc, b->st_q, b->st_id, b->st_side,
                  b->st_lam, b->st_qr, b->fw_status, b->fw_nu};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete b;
}

// Fork the batch's side streams from `stream` (they wait for everything
// queued on it so far); true when there are side streams and it worked.
bool fork_lanes(rbp_batch* b, hipStream_t stream) {
  if (b->groups.size() <= 1 || !b->ev_fork) return false;
  if (hipEventRecord(b->ev_fork, stream) != hipSuccess) return false;
  for (int l = 0; l < rbp_batch::kLanes - 1; ++l)
    if (hipStreamWaitEvent(b->side[l], b->ev_fork, 0) != hipSuccess) return false;
  return true;
}
// Join the side streams back into `stream` (it waits for their work).
bool join_lanes(rbp_batch* b, hipStream_t stream) {
  for (int l = 0; l < rbp_batch::kLanes - 1; ++l)
    if (hipEventRecord(b->ev_join[l], b->side[l]) != hipSuccess ||
        hipStreamWaitEvent(stream, b->ev_join[l], 0) != hipSuccess)
      return false;
  return true;
}
hipStream_t lane_stream(const rbp_batch* b, size_t group, hipStream_t stream) {
  const int l = b->groups.size() > 1 ? b->group_lane[group] : 0;
  return l == 0 ? stream : b->side[l - 1];
}

template <typename T>
int d2h(std::vector<T>& dst, const T* src, size_t n, hipStream_t s) {
  dst.resize(n);
  if (n == 0) return RBP_OK;
  if (hipMemcpyAsync(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, s) != hipSuccess) return RBP_E_DEVICE;
  return RBP_OK;
}

}  // namespace

extern "C" {

void rbp_default_opts(rbp_solve_opts* o) {
  if (!o) return;
  o->admm_iters = 10;
  o->rho = 0.1f;
  o->alpha = 1.6f;
  o->max_polish_steps = 0;
  o->feas_tol = 1e-11;
  o->kkt_tol = 1e-6;
  o->store_for_backward = 1;
  o->plain = 0;
  o->launch_shape = 0;
  o->schedule = 0;
  o->debug_fill_lds = 0;
  o->reserved = 0;
}

const char* rbp_status_string(int code) {
  switch (code) {
    case 0: return "ok / solved";
    case RBP_INFEASIBLE: return "infeasible (verified certificate)";
    case RBP_MAXITER: return "iteration limit";
    case RBP_POLISH_FAILED: return "polish failed";
    case RBP_NUMERICAL: return "numerical: KKT tolerance missed";
    case RBP_INVALID_INPUT: return "invalid instance input";
    case RBP_E_INVALID: return "invalid argument";
    case RBP_E_SHAPE: return "inconsistent shapes or offsets";
    case RBP_E_ALLOC: return "device allocation failed";
    case RBP_E_DEVICE: return "HIP runtime error";
    case RBP_E_STATE: return "no stored forward pass";
    case RBP_E_SCRATCH: return "problem larger than the fixed workspace of an allocation-free call";
    default: return "unknown code";
  }
}

int rbp_build_batch(const rbp_problem_desc* d, hipStream_t stream, rbp_batch** out) {
  if (!d || !out) return RBP_E_INVALID;
  *out = nullptr;
  const int32_t N = d->n_instances;
  if (N < 0 || d->n_poly < 0) return RBP_E_INVALID;
  if (!(d->vmax > 0.0) || !(d->amax > 0.0)) return RBP_E_INVALID;
  if (d->pin_start_velocity != 0 && d->pin_start_velocity != 1) return RBP_E_INVALID;
  if (N > 0) {
    if (d->n_poly < 1) return RBP_E_SHAPE;
    if (!d->degree || !d->T || !d->poly_off || !d->A_face || !d->b_face || !d->poly_idx ||
        !d->reach_off || !d->H_off || !d->H || !d->h0 || !d->G)
      return RBP_E_INVALID;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RBP_E_DEVICE;
  {
    // the device's side streams are made at the first batch, whatever its
    // groups, so that they are among the process's first streams
    hipStream_t early[3];
    if (!side_streams(dev, early)) return RBP_E_DEVICE;
  }
  if (int rc = ensure_constants(dev)) return rc;

  // reachable blocks: one per instance, or a shared table indexed by reach_idx
  const bool shared_reach = d->reach_idx != nullptr;
  if (N > 0 && shared_reach && d->n_reach < 1) return RBP_E_SHAPE;
  const size_t n_blk = shared_reach ? size_t(d->n_reach) : size_t(N);
  std::vector<int32_t> deg, pidx, poff, ridx;
  std::vector<int64_t> roff, hoff;
  int rc = RBP_OK;
  if (N > 0) {
    if ((rc = d2h(deg, d->degree, N, stream)) || (rc = d2h(pidx, d->poly_idx, N, stream)) ||
        (rc = d2h(poff, d->poly_off, size_t(d->n_poly) + 1, stream)) ||
        (rc = d2h(roff, d->reach_off, n_blk + 1, stream)) || (rc = d2h(hoff, d->H_off, n_blk + 1, stream)) ||
        (shared_reach && (rc = d2h(ridx, d->reach_idx, N, stream))))
      return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return RBP_E_DEVICE;
  }
  auto blk = [&](int i) -> int { return shared_reach ? ridx[i] : i; };
  auto* b = new (std::nothrow) rbp_batch();
  if (!b) return RBP_E_ALLOC;
  b->device = dev;
  b->desc = *d;
  b->N = N;
  std::vector<int64_t> pt_off(size_t(N) + 1, 0), face_off(size_t(N) + 1, 0);
  std::vector<int32_t> order(N);
  if (N > 0) {
    if (poff[0] != 0) { free_batch(b); return RBP_E_SHAPE; }
    for (int j = 0; j < d->n_poly; ++j) {
      const int64_t nf = int64_t(poff[j + 1]) - poff[j];
      if (nf < 1 || nf > RBP_MAX_FACES) { free_batch(b); return RBP_E_SHAPE; }
    }
    if (roff[0] != 0 || hoff[0] != 0) { free_batch(b); return RBP_E_SHAPE; }
    std::vector<int64_t> cost(N);
    for (int i = 0; i < N; ++i) {
      const int p = deg[i];
      if (p < RBP_MIN_DEGREE || p > RBP_MAX_DEGREE) { free_batch(b); return RBP_E_SHAPE; }
      if (pidx[i] < 0 || pidx[i] >= d->n_poly) { free_batch(b); return RBP_E_SHAPE; }
      const int k = blk(i);
      if (k < 0 || size_t(k) >= n_blk) { free_batch(b); return RBP_E_SHAPE; }
      const int64_t r = roff[k + 1] - roff[k];
      if (r < 0 || r > RBP_MAX_REACH) { free_batch(b); return RBP_E_SHAPE; }
      if (hoff[k + 1] - hoff[k] != r * 3 * (p + 1)) { free_batch(b); return RBP_E_SHAPE; }
      const int nf = poff[pidx[i] + 1] - poff[pidx[i]];
      b->pmax = std::max<int32_t>(b->pmax, p);
      b->rmax = std::max<int32_t>(b->rmax, int32_t(r));
      b->nfmax = std::max<int32_t>(b->nfmax, nf);
      pt_off[i + 1] = pt_off[i] + (p + 1);
      face_off[i + 1] = face_off[i] + nf;
      cost[i] = int64_t(3 * (p - 1)) * ((p - 1) * nf + 6 * p + r);
    }
    b->F_total = poff[d->n_poly];
    // work order: grouped by degree and reachable-row class (one specialised
    // launch each, LDS sized per group), most expensive first within a group
    // so that the tail of each launch is short
    auto rclass = [&](int i) -> int {
      const int64_t r = roff[blk(i) + 1] - roff[blk(i)];
      return r <= 32 ? 0 : (r <= 64 ? 1 : 2);
    };
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
      if (deg[a] != deg[c]) return deg[a] < deg[c];
      const int ra = rclass(a), rc2 = rclass(c);
      return ra != rc2 ? ra < rc2 : cost[a] > cost[c];
    });
    // estimated work of a group: its instances' cost, scaled by how few of
    // its workgroups fit a CU (a group of large instances runs at low
    // residency, so each instance takes longer)
    std::vector<int64_t> gcost;
    for (int k = 0; k < N; ++k) {
      const int i = order[k];
      const int32_t r = int32_t(roff[blk(i) + 1] - roff[blk(i)]);
      const int32_t nf = poff[pidx[i] + 1] - poff[pidx[i]];
      if (b->groups.empty() || b->groups.back().p != deg[i] || rclass(order[b->groups.back().start]) != rclass(i)) {
        b->groups.push_back({deg[i], k, 0, 0, 1});
        gcost.push_back(0);
      }
      rbp_batch::Group& g = b->groups.back();
      ++g.count;
      g.rmax = std::max(g.rmax, r);
      g.nfmax = std::max(g.nfmax, nf);
      gcost.back() += cost[i];
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      const rbp_batch::Group& g = b->groups[gi];
      const size_t bytes = size_t(rbp::make_dims(g.p, g.rmax, g.nfmax, 4, false).bytes);
      const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, int64_t(kLdsBytes / std::max<size_t>(bytes, 1))));
      gcost[gi] = gcost[gi] * 8 / per_cu;
    }
    b->degree_host = deg;
    // streams of the groups: longest processing time first onto the least
    // loaded stream, and launched in that order (each stream starts with its
    // longest group)
    b->group_lane.assign(b->groups.size(), 0);
    b->launch_order.resize(b->groups.size());
    std::iota(b->launch_order.begin(), b->launch_order.end(), 0);
    std::stable_sort(b->launch_order.begin(), b->launch_order.end(),
                     [&](int x, int y) { return gcost[size_t(x)] > gcost[size_t(y)]; });
    if (b->groups.size() > 1) {
      const std::vector<int32_t>& byc = b->launch_order;
      int64_t load[rbp_batch::kLanes] = {};
      for (int gi : byc) {
        int best = 0;
        for (int l = 1; l < rbp_batch::kLanes; ++l)
          if (load[l] < load[best]) best = l;
        b->group_lane[size_t(gi)] = best;
        load[best] += gcost[size_t(gi)];
      }
      bool ok = side_streams(dev, b->side) &&
                hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) == hipSuccess;
      for (int l = 0; ok && l < rbp_batch::kLanes - 1; ++l)
        ok = hipEventCreateWithFlags(&b->ev_join[l], hipEventDisableTiming) == hipSuccess;
      if (!ok) { free_batch(b); return RBP_E_DEVICE; }
    }
  }
  // descriptors in work-order position and the inverse permutation
  std::vector<rbp::InstDesc> desc(static_cast<size_t>(N));
  b->pos_host.assign(size_t(N), 0);
  for (int k = 0; k < N; ++k) {
    const int i = order[k];
    const int blk_i = blk(i);
    rbp::InstDesc& q = desc[size_t(k)];
    q.inst = i;
    q.p = deg[i];
    q.f0 = poff[pidx[i]];
    q.nf = poff[pidx[i] + 1] - poff[pidx[i]];
    q.r = int32_t(roff[blk_i + 1] - roff[blk_i]);
    q.pad0 = 0;
    q.r0 = roff[blk_i];
    q.hb = hoff[blk_i];
    q.po = pt_off[i];
    q.fo = face_off[i];
    q.pad1 = 0;
    b->pos_host[size_t(i)] = k;
  }
  b->pt_total = pt_off[N];
  b->face_total = face_off[N];
  b->nmax = 3 * (b->pmax - 1);
  const size_t n1 = size_t(N);
  if ((rc = dalloc(&b->d_pt_off, n1 + 1)) || (rc = dalloc(&b->d_face_off, n1 + 1)) ||
      (rc = dalloc(&b->d_order, n1)) || (rc = dalloc(&b->d_desc, n1)) || (rc = dalloc(&b->st_q, n1)) ||
      (rc = dalloc(&b->st_id, n1 * b->nmax)) || (rc = dalloc(&b->st_side, n1 * b->nmax)) ||
      (rc = dalloc(&b->st_lam, n1 * b->nmax)) || (rc = dalloc(&b->st_qr, n1 * 2 * b->nmax * b->nmax)) ||
      (rc = dalloc(&b->fw_status, n1)) || (rc = dalloc(&b->fw_nu, 6 * n1))) {
    free_batch(b);
    return rc;
  }
  if (hipMemcpyAsync(b->d_pt_off, pt_off.data(), (n1 + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream) ||
      hipMemcpyAsync(b->d_face_off, face_off.data(), (n1 + 1) * sizeof(int64_t), hipMemcpyHostToDevice, stream) ||
      (N > 0 && hipMemcpyAsync(b->d_order, order.data(), n1 * sizeof(int32_t), hipMemcpyHostToDevice, stream)) ||
      (N > 0 && hipMemcpyAsync(b->d_desc, desc.data(), n1 * sizeof(rbp::InstDesc), hipMemcpyHostToDevice, stream)) ||
      hipStreamSynchronize(stream)) {
    free_batch(b);
    return RBP_E_DEVICE;
  }
  b->last_stream = stream;
  *out = b;
  return RBP_OK;
}

int rbp_batch_get_sizes(const rbp_batch* b, rbp_batch_sizes* out) {
  if (!b || !out) return RBP_E_INVALID;
  out->n_instances = b->N;
  out->max_degree = b->pmax;
  out->points_total = b->pt_total;
  out->faces_total = b->face_total;
  return RBP_OK;
}

int rbp_solve_batch(rbp_batch* b, const double* x0, const double* goal, const double* b_face,
                    const rbp_solve_opts* opts_in, double* P_out, double* cost_out, int32_t* status_out,
                    double* kkt_out, int32_t* iters_out, hipStream_t stream) {
  if (!b) return RBP_E_INVALID;
  rbp_solve_opts o;
  rbp_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.admm_iters < 0 || !(o.rho > 0.0f) || !(o.alpha > 0.0f) || !(o.alpha < 2.0f) || o.max_polish_steps < 0 ||
      !(o.feas_tol > 0.0) || !(o.kkt_tol > 0.0) || o.launch_shape < 0 || o.launch_shape > 2 ||
      o.schedule < 0 || o.schedule > 1 || o.debug_fill_lds < 0 || o.debug_fill_lds > 1 || o.reserved != 0)
    return RBP_E_INVALID;
  b->has_forward = false;
  if (b->N == 0) return RBP_OK;
  if (!x0 || !goal || !P_out || !cost_out || !status_out || !kkt_out) return RBP_E_INVALID;
  const rbp_problem_desc& d = b->desc;
  const double* bf = b_face ? b_face : d.b_face;

  rbp::SolveArgs a{};
  a.N = b->N;
  a.degree = d.degree; a.T = d.T; a.poly_off = d.poly_off; a.A_face = d.A_face; a.b_face = bf;
  a.poly_idx = d.poly_idx; a.reach_off = d.reach_off; a.H_off = d.H_off; a.H = d.H; a.h0 = d.h0; a.G = d.G;
  a.reach_idx = d.reach_idx;
  a.pin_v0 = d.pin_start_velocity;
  a.vmax = d.vmax; a.amax = d.amax;
  a.x0 = x0; a.goal = goal; a.pt_off = b->d_pt_off;
  a.P_out = P_out; a.cost_out = cost_out; a.status_out = status_out; a.kkt_out = kkt_out; a.iters_out = iters_out;
  a.store = o.store_for_backward ? 1 : 0;
  a.debug_fill = o.debug_fill_lds;
  if (a.store) { a.fw_status = b->fw_status; a.fw_nu = b->fw_nu; }
  a.st_q = b->st_q; a.st_id = b->st_id; a.st_side = b->st_side; a.st_lam = b->st_lam; a.st_qr = b->st_qr;
  a.st_stride = b->nmax;
  a.admm_iters = o.admm_iters; a.rho = o.rho; a.alpha = o.alpha;
  a.max_steps = o.max_polish_steps; a.feas_tol = o.feas_tol; a.kkt_tol = o.kkt_tol;
  hipError_t e = hipSuccess;
  a.desc = b->d_desc;
  if (o.plain) {
    a.order = b->d_order;
    a.dims = rbp::make_dims(b->pmax, b->rmax, b->nfmax, 8, o.admm_iters > 0);
    for (int i = 0; i < b->N && e == hipSuccess; ++i) {
      a.inst_base = b->pos_host[size_t(i)];
      a.N = a.inst_base + 1;
      e = rbp::launch_solve(a, 1, stream, true, b->degree_host[i]);
    }
  } else if (o.schedule == 1) {
    a.order = b->d_order;
    a.dims = rbp::make_dims(b->pmax, b->rmax, b->nfmax, 4, o.admm_iters > 0);
    a.inst_base = 0;
    a.N = b->N;
    e = rbp::launch_solve_all(a, b->N, stream);
  } else {
    a.order = b->d_order;
    const bool fork = fork_lanes(b, stream);
    if (b->groups.size() > 1 && !fork) return RBP_E_DEVICE;
    for (size_t j = 0; j < b->groups.size() && e == hipSuccess; ++j) {
      const size_t k = size_t(b->launch_order[j]);
      const rbp_batch::Group& g = b->groups[k];
      const hipStream_t gs = lane_stream(b, k, stream);
      a.dims = rbp::make_dims(g.p, g.rmax, g.nfmax, 4, o.admm_iters > 0);
      a.inst_base = g.start;
      a.N = g.start + g.count;
      // two instances per workgroup only while both slices fit the LDS
      int shape = o.launch_shape;
      if (rbp::kShapeWaves[shape] * size_t(a.dims.bytes) > kLdsBytes) shape = rbp::kShapeW1E2;
      e = shape == rbp::kShapeW1E2 ? rbp::launch_solve(a, g.count, gs, false, g.p)
                                   : rbp::launch_solve_shape(a, g.count, gs, g.p, shape);
    }
    if (fork && !join_lanes(b, stream) && e == hipSuccess) e = hipErrorUnknown;
  }
  if (e != hipSuccess) return RBP_E_DEVICE;
  b->last_stream = stream;
  b->fw_schedule = o.schedule;
  b->fw_debug_fill = o.debug_fill_lds;
  if (o.store_for_backward) b->has_forward = true;
  return RBP_OK;
}

int rbp_backward(rbp_batch* b, const double* grad_P, const double* grad_cost, double* grad_x0, double* grad_goal,
                 double* grad_b, int32_t* flags_out, hipStream_t stream) {
  if (!b) return RBP_E_INVALID;
  if (!b->has_forward) return RBP_E_STATE;
  if (b->N == 0) return RBP_OK;
  if (!grad_x0 || !grad_goal || !grad_b) return RBP_E_INVALID;
  const rbp_problem_desc& d = b->desc;
  rbp::BackArgs a{};
  a.N = b->N;
  a.degree = d.degree; a.T = d.T; a.poly_off = d.poly_off; a.A_face = d.A_face;
  a.poly_idx = d.poly_idx; a.reach_off = d.reach_off; a.H_off = d.H_off; a.H = d.H; a.G = d.G;
  a.reach_idx = d.reach_idx;
  a.pin_v0 = d.pin_start_velocity;
  a.vmax = d.vmax; a.amax = d.amax;
  a.nu = b->fw_nu; a.pt_off = b->d_pt_off; a.face_off = b->d_face_off;
  a.status = b->fw_status;
  a.st_q = b->st_q; a.st_id = b->st_id; a.st_side = b->st_side; a.st_lam = b->st_lam; a.st_qr = b->st_qr;
  a.grad_P = grad_P; a.grad_cost = grad_cost;
  a.grad_x0 = grad_x0; a.grad_goal = grad_goal; a.grad_b = grad_b; a.flags = flags_out;
  a.order = b->d_order;
  a.desc = b->d_desc;
  a.st_stride = b->nmax;
  a.debug_fill = b->fw_debug_fill;
  if (b->fw_schedule == 1) {
    a.dims = rbp::make_back_dims(b->pmax, b->nfmax);
    a.inst_base = 0;
    if (rbp::launch_backward_all(a, b->N, stream) != hipSuccess) return RBP_E_DEVICE;
    b->last_stream = stream;
    return RBP_OK;
  }
  const bool fork = fork_lanes(b, stream);
  if (b->groups.size() > 1 && !fork) return RBP_E_DEVICE;
  hipError_t e = hipSuccess;
  for (size_t j = 0; j < b->groups.size() && e == hipSuccess; ++j) {
    const size_t k = size_t(b->launch_order[j]);
    const rbp_batch::Group& g = b->groups[k];
    a.dims = rbp::make_back_dims(g.p, g.nfmax);
    a.inst_base = g.start;
    a.N = g.start + g.count;
    e = rbp::launch_backward(a, g.count, lane_stream(b, k, stream), g.p);
  }
  if (fork && !join_lanes(b, stream) && e == hipSuccess) e = hipErrorUnknown;
  if (e != hipSuccess) return RBP_E_DEVICE;
  b->last_stream = stream;
  return RBP_OK;
}

struct rbp_chains {
  int device = 0;
  rbp_chain_desc desc{};
  int32_t N = 0, s_max = 1, nf_max = 1, r_max = 0;
  int64_t pt_total = 0;
  int32_t* d_order = nullptr;
  int32_t* ws_keys = nullptr;   // working set of each path at its first-pass overflow
  int32_t* ws_meta = nullptr;   // its row count and the polish steps taken
  // work order, most segments first (longest paths start first, so a
  // launch's tail is short); launch groups by ranges of segment counts, each
  // with its own LDS size, run on kLanes streams at once (the caller's and
  // the device's kLanes - 1 side streams, forked and joined with events),
  // assigned longest estimated work first to the least loaded stream
  struct Group { int32_t start, count, s_max, nf_max, r_max; };
  std::vector<Group> groups;
  static constexpr int kLanes = 4;
  std::vector<int32_t> group_lane;
  hipStream_t side[kLanes - 1] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kLanes - 1] = {};
  hipStream_t last_stream = nullptr;
};

namespace {
std::vector<int> g_chain_const_done;
int ensure_chain_constants(int device) {
  std::lock_guard<std::mutex> lk(g_const_mu);
  if (std::find(g_chain_const_done.begin(), g_chain_const_done.end(), device) != g_chain_const_done.end())
    return RBP_OK;
  if (rbp::upload_chain_constants(device) != hipSuccess) return RBP_E_DEVICE;
  g_chain_const_done.push_back(device);
  return RBP_OK;
}
// working-set capacity of the path polish: two entries per lane (at most
// 127 rows).  The dual method keeps linearly independent normals, so a path
// with n free variables never holds more than n; the polish stops when q
// reaches the capacity minus one, hence n + 2 for short paths.
// working-set rows of the first path pass: at 12 segments of degree 7 its LDS
// (about 50 KB) leaves three paths resident per CU, against one at the full cap
constexpr int kChainFirstPassRows = 32;

void free_chains(rbp_chains* c) {
  for (int k = 0; k < rbp_chains::kLanes - 1; ++k) {
    if (c->side[k]) (void)hipStreamSynchronize(c->side[k]);   // shared: not destroyed
    if (c->ev_join[k]) (void)hipEventDestroy(c->ev_join[k]);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  for (int32_t* p : {c->d_order, c->ws_keys, c->ws_meta})
    if (p) (void)hipFree(p);
  delete c;
}

// launch groups of a path batch by segment count (S >= 12, 10-11, 8-9, 6-7,
// up to 5): each group's LDS is sized for its longest path, so short paths
// are resident four to a CU.  On the 8,192-path batch (4-12 segments) this
// took 29.3 ms against 31.5 ms for one group; one group per count (34.9 ms)
// or per three counts (33.7 ms) was slower: the groups share four streams,
// and a stream waits out each of its groups' full-cap tails in turn.
constexpr int kChainGroupMinS[] = {12, 10, 8, 6, 1};
int chain_bucket(int S) {
  int k = 0;
  while (S < kChainGroupMinS[k]) ++k;
  return k;
}

int chain_q_cap(int p, int s_max) {
  const int n = 3 * ((p - 1) + (s_max - 1) * (p - 2));
  return std::min(128, n + 2);
}
}  // namespace

int rbp_build_chains(const rbp_chain_desc* d, hipStream_t stream, rbp_chains** out) {
  if (!d || !out) return RBP_E_INVALID;
  *out = nullptr;
  const int32_t N = d->n_chains;
  if (N < 0 || d->n_poly < 0 || !(d->T > 0.0) || !(d->vmax > 0.0) || !(d->amax > 0.0)) return RBP_E_INVALID;
  if (d->degree != RBP_CHAIN_DEGREE) return RBP_E_SHAPE;
  if (N > 0 && (!d->seg_off || !d->poly_off || !d->A_face || !d->b_face || !d->poly_idx || !d->reach_off ||
                !d->H_off || !d->H || !d->h0 || !d->G))
    return RBP_E_INVALID;
  if (N > 0 && d->n_poly < 1) return RBP_E_SHAPE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RBP_E_DEVICE;
  {
    // the device's side streams are made at the first batch, whatever its
    // groups, so that they are among the process's first streams
    hipStream_t early[3];
    if (!side_streams(dev, early)) return RBP_E_DEVICE;
  }
  if (int rc = ensure_chain_constants(dev)) return rc;
  std::vector<int64_t> soff;
  int rc = RBP_OK;
  if (N > 0) {
    if ((rc = d2h(soff, d->seg_off, size_t(N) + 1, stream))) return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return RBP_E_DEVICE;
    if (soff[0] != 0) return RBP_E_SHAPE;
  }
  const int64_t nseg = N > 0 ? soff[N] : 0;
  std::vector<int32_t> pidx, poff;
  std::vector<int64_t> roff, hoff;
  if (N > 0) {
    if ((rc = d2h(pidx, d->poly_idx, size_t(nseg), stream)) || (rc = d2h(poff, d->poly_off, size_t(d->n_poly) + 1, stream)) ||
        (rc = d2h(roff, d->reach_off, size_t(nseg) + 1, stream)) || (rc = d2h(hoff, d->H_off, size_t(nseg) + 1, stream)))
      return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return RBP_E_DEVICE;
  }
  auto* c = new (std::nothrow) rbp_chains();
  if (!c) return RBP_E_ALLOC;
  c->device = dev;
  c->desc = *d;
  c->N = N;
  const int p = d->degree;
  std::vector<int32_t> order(N);
  if (N > 0) {
    if (poff[0] != 0 || roff[0] != 0 || hoff[0] != 0) { delete c; return RBP_E_SHAPE; }
    for (int j = 0; j < d->n_poly; ++j) {
      const int nf = poff[j + 1] - poff[j];
      if (nf < 1 || nf > RBP_MAX_FACES) { delete c; return RBP_E_SHAPE; }
    }
    for (int i = 0; i < N; ++i) {
      const int64_t S = soff[i + 1] - soff[i];
      if (S < 1 || S > RBP_CHAIN_MAX_SEGMENTS) { delete c; return RBP_E_SHAPE; }
      c->s_max = std::max<int32_t>(c->s_max, int32_t(S));
    }
    for (int64_t s = 0; s < nseg; ++s) {
      if (pidx[s] < 0 || pidx[s] >= d->n_poly) { delete c; return RBP_E_SHAPE; }
      const int64_t r = roff[s + 1] - roff[s];
      if (r < 0 || r > RBP_MAX_REACH || hoff[s + 1] - hoff[s] != r * 3 * (p + 1)) { delete c; return RBP_E_SHAPE; }
      c->r_max = std::max<int32_t>(c->r_max, int32_t(r));
      c->nf_max = std::max<int32_t>(c->nf_max, poff[pidx[s] + 1] - poff[pidx[s]]);
    }
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return soff[a + 1] - soff[a] > soff[b + 1] - soff[b];
    });
    // estimated work of a path: its polish steps and the cost of one both
    // grow with its segment count
    std::vector<int64_t> gcost;
    for (int k = 0; k < N; ++k) {
      const int i = order[k];
      const int32_t S = int32_t(soff[i + 1] - soff[i]);
      if (c->groups.empty() || chain_bucket(c->groups.back().s_max) != chain_bucket(S)) {
        c->groups.push_back({k, 0, S, 1, 0});
        gcost.push_back(0);
      }
      rbp_chains::Group& g = c->groups.back();
      ++g.count;
      g.s_max = std::max(g.s_max, S);
      gcost.back() += int64_t(S) * S;
      for (int64_t s = soff[i]; s < soff[i + 1]; ++s) {
        g.r_max = std::max<int32_t>(g.r_max, int32_t(roff[s + 1] - roff[s]));
        g.nf_max = std::max<int32_t>(g.nf_max, poff[pidx[s] + 1] - poff[pidx[s]]);
      }
    }
    c->group_lane.assign(c->groups.size(), 0);
    if (c->groups.size() > 1) {
      std::vector<int> byc(c->groups.size());
      std::iota(byc.begin(), byc.end(), 0);
      std::stable_sort(byc.begin(), byc.end(), [&](int x, int y) { return gcost[size_t(x)] > gcost[size_t(y)]; });
      int64_t load[rbp_chains::kLanes] = {};
      for (int gi : byc) {
        int best = 0;
        for (int l = 1; l < rbp_chains::kLanes; ++l)
          if (load[l] < load[best]) best = l;
        c->group_lane[size_t(gi)] = best;
        load[best] += gcost[size_t(gi)];
      }
      bool ok = side_streams(dev, c->side) &&
                hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess;
      for (int l = 0; ok && l < rbp_chains::kLanes - 1; ++l)
        ok = hipEventCreateWithFlags(&c->ev_join[l], hipEventDisableTiming) == hipSuccess;
      if (!ok) { free_chains(c); return RBP_E_DEVICE; }
    }
  }
  c->pt_total = int64_t(p + 1) * nseg;
  const size_t n1 = size_t(std::max(N, 1));
  if ((rc = dalloc(&c->d_order, n1)) || (rc = dalloc(&c->ws_keys, n1 * kChainFirstPassRows)) ||
      (rc = dalloc(&c->ws_meta, 2 * n1))) {
    free_chains(c);
    return rc;
  }
  if (N > 0 && (hipMemcpyAsync(c->d_order, order.data(), size_t(N) * 4, hipMemcpyHostToDevice, stream) ||
                hipStreamSynchronize(stream))) {
    free_chains(c);
    return RBP_E_DEVICE;
  }
  c->last_stream = stream;
  *out = c;
  return RBP_OK;
}

int rbp_chains_get_sizes(const rbp_chains* c, rbp_batch_sizes* out) {
  if (!c || !out) return RBP_E_INVALID;
  out->n_instances = c->N;
  out->max_degree = c->desc.degree;
  out->points_total = c->pt_total;
  out->faces_total = 0;
  return RBP_OK;
}

int rbp_solve_chains(rbp_chains* c, const double* x0, const double* goal, const rbp_solve_opts* opts_in,
                     double* P_out, double* cost_out, int32_t* status_out, double* kkt_out, int32_t* iters_out,
                     hipStream_t stream) {
  if (!c) return RBP_E_INVALID;
  rbp_solve_opts o;
  rbp_default_opts(&o);
  if (opts_in) o = *opts_in;
  if (o.admm_iters < 0 || !(o.rho > 0.0f) || !(o.alpha > 0.0f) || !(o.alpha < 2.0f) || o.max_polish_steps < 0 ||
      !(o.feas_tol > 0.0) || !(o.kkt_tol > 0.0))
    return RBP_E_INVALID;
  if (c->N == 0) return RBP_OK;
  if (!x0 || !goal || !P_out || !cost_out || !status_out || !kkt_out) return RBP_E_INVALID;
  const rbp_chain_desc& d = c->desc;
  rbp::ChainArgs a{};
  a.N = c->N; a.P = d.degree; a.T = d.T; a.vmax = d.vmax; a.amax = d.amax;
  a.seg_off = d.seg_off; a.poly_off = d.poly_off; a.A_face = d.A_face; a.b_face = d.b_face;
  a.poly_idx = d.poly_idx; a.reach_off = d.reach_off; a.H_off = d.H_off; a.H = d.H; a.h0 = d.h0; a.G = d.G;
  a.x0 = x0; a.goal = goal; a.order = c->d_order;
  a.ws_keys = c->ws_keys; a.ws_meta = c->ws_meta; a.ws_stride = kChainFirstPassRows;
  a.P_out = P_out; a.cost_out = cost_out; a.status_out = status_out; a.kkt_out = kkt_out; a.iters_out = iters_out;
  a.admm_iters = o.admm_iters; a.rho = o.rho; a.alpha = o.alpha; a.max_steps = o.max_polish_steps;
  a.feas_tol = o.feas_tol; a.kkt_tol = o.kkt_tol;
  // fork the side streams from the caller's (they wait for its queued work),
  // launch every group on its stream, join them back into the caller's
  const bool fork = c->groups.size() > 1 && c->ev_fork;
  if (fork) {
    if (hipEventRecord(c->ev_fork, stream) != hipSuccess) return RBP_E_DEVICE;
    for (int l = 0; l < rbp_chains::kLanes - 1; ++l)
      if (hipStreamWaitEvent(c->side[l], c->ev_fork, 0) != hipSuccess) return RBP_E_DEVICE;
  }
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < c->groups.size() && e == hipSuccess; ++k) {
    const rbp_chains::Group& g = c->groups[k];
    const int l = fork ? c->group_lane[k] : 0;
    const hipStream_t gs = l == 0 ? stream : c->side[l - 1];
    // a first pass with a small working-set cap keeps LDS per path low (more
    // paths resident per CU); the few paths whose working set outgrows it are
    // finished by a full-cap pass, which continues from the working set the
    // first pass held and skips every other path
    const int q_full = chain_q_cap(d.degree, g.s_max);
    const int q_first = std::min(q_full, kChainFirstPassRows);
    const bool admm = o.admm_iters > 0;
    a.inst_base = g.start;
    a.N = g.start + g.count;
    a.q_full = q_full;
    a.retry_only = 0;
    a.dims = rbp::make_chain_dims(d.degree, g.s_max, g.nf_max, g.r_max, q_first, admm);
    e = rbp::launch_chains(a, gs);
    if (e == hipSuccess && q_first < q_full) {
      a.retry_only = 1;
      a.dims = rbp::make_chain_dims(d.degree, g.s_max, g.nf_max, g.r_max, q_full, admm);
      e = rbp::launch_chains(a, gs);
    }
  }
  if (fork)
    for (int l = 0; l < rbp_chains::kLanes - 1; ++l)
      if (hipEventRecord(c->ev_join[l], c->side[l]) != hipSuccess ||
          hipStreamWaitEvent(stream, c->ev_join[l], 0) != hipSuccess)
        e = e == hipSuccess ? hipErrorUnknown : e;
  if (e != hipSuccess) return RBP_E_DEVICE;
  c->last_stream = stream;
  return RBP_OK;
}

void rbp_destroy_chains(rbp_chains* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->last_stream) (void)hipStreamSynchronize(c->last_stream);
  free_chains(c);
}

void rbp_destroy_batch(rbp_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  if (b->last_stream) (void)hipStreamSynchronize(b->last_stream);
  else (void)hipDeviceSynchronize();
  free_batch(b);
}

struct rbp_cut {
  int device = 0;
  rbp_cut_desc desc{};
  unsigned long long* counter = nullptr;
  int64_t* list = nullptr;
  int64_t cap = 0;
  int qp_blocks = 0;
  int32_t* pv_off = nullptr;    // vertex table of the polytope obstacles
  double* pv = nullptr;
  hipStream_t last_stream = nullptr;
};

namespace {
void free_cut(rbp_cut* c) {
  for (void* p : {static_cast<void*>(c->counter), static_cast<void*>(c->list), static_cast<void*>(c->pv_off),
                  static_cast<void*>(c->pv)})
    if (p) (void)hipFree(p);
  delete c;
}

// Vertices of {x : a_k . x <= b_k, k < m} in R^3: every intersection point of
// three planes with independent normals that satisfies all rows (to a
// relative 1e-9), points closer than that merged.  Appends to `out` and
// returns the count, or -1 past `cap`.
int polytope_vertices(const double* A, const double* b, int m, int cap, std::vector<double>& out) {
  const size_t base = out.size();
  double scale = 1.0;
  for (int k = 0; k < m; ++k) scale = std::max(scale, std::fabs(b[k]));
  int count = 0;
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j)
      for (int k = j + 1; k < m; ++k) {
        const double* a0 = A + 3 * i;
        const double* a1 = A + 3 * j;
        const double* a2 = A + 3 * k;
        // Cramer's rule: x = (b_i (a1 x a2) + b_j (a2 x a0) + b_k (a0 x a1)) / det
        const double c12[3] = {a1[1] * a2[2] - a1[2] * a2[1], a1[2] * a2[0] - a1[0] * a2[2], a1[0] * a2[1] - a1[1] * a2[0]};
        const double c20[3] = {a2[1] * a0[2] - a2[2] * a0[1], a2[2] * a0[0] - a2[0] * a0[2], a2[0] * a0[1] - a2[1] * a0[0]};
        const double c01[3] = {a0[1] * a1[2] - a0[2] * a1[1], a0[2] * a1[0] - a0[0] * a1[2], a0[0] * a1[1] - a0[1] * a1[0]};
        const double det = a0[0] * c12[0] + a0[1] * c12[1] + a0[2] * c12[2];
        const double n0 = std::sqrt(a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2]);
        const double n1 = std::sqrt(a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2]);
        const double n2 = std::sqrt(a2[0] * a2[0] + a2[1] * a2[1] + a2[2] * a2[2]);
        if (!(std::fabs(det) > 1e-10 * n0 * n1 * n2)) continue;
        double x[3];
        for (int c = 0; c < 3; ++c) x[c] = (b[i] * c12[c] + b[j] * c20[c] + b[k] * c01[c]) / det;
        bool ok = true;
        for (int r = 0; r < m && ok; ++r) {
          const double* ar = A + 3 * r;
          const double nr = std::sqrt(ar[0] * ar[0] + ar[1] * ar[1] + ar[2] * ar[2]);
          ok = ar[0] * x[0] + ar[1] * x[1] + ar[2] * x[2] <= b[r] + 1e-9 * nr * scale;
        }
        if (!ok) continue;
        bool dup = false;
        for (int v = 0; v < count && !dup; ++v) {
          const double* y = out.data() + base + 3 * v;
          dup = std::fabs(x[0] - y[0]) <= 1e-9 * scale && std::fabs(x[1] - y[1]) <= 1e-9 * scale &&
                std::fabs(x[2] - y[2]) <= 1e-9 * scale;
        }
        if (dup) continue;
        if (count >= cap) return -1;
        out.insert(out.end(), x, x + 3);
        ++count;
      }
  return count;
}

// A polytope {A x <= b} is bounded exactly when its recession cone
// {d : A d <= 0} is {0}: the vertices of that cone cut by the cube
// |d_i| <= 1 are then only the origin.
bool polytope_bounded(const double* A, int m) {
  std::vector<double> Ab(size_t(3 * (m + 6)), 0.0), bb(size_t(m + 6), 0.0);
  std::copy(A, A + 3 * m, Ab.begin());
  for (int c = 0; c < 3; ++c) {
    Ab[size_t(3 * (m + 2 * c) + c)] = 1.0;
    bb[size_t(m + 2 * c)] = 1.0;
    Ab[size_t(3 * (m + 2 * c + 1) + c)] = -1.0;
    bb[size_t(m + 2 * c + 1)] = 1.0;
  }
  std::vector<double> v;
  const int n = polytope_vertices(Ab.data(), bb.data(), m + 6, 4096, v);
  if (n < 0) return false;
  for (double x : v)
    if (std::fabs(x) > 1e-7) return false;
  return true;
}
}  // namespace

int rbp_build_cut(const rbp_cut_desc* d, hipStream_t stream, rbp_cut** out) {
  if (!d || !out) return RBP_E_INVALID;
  *out = nullptr;
  if (d->n_edges < 0 || d->n_obstacles < 0 || d->reserved != 0 || d->n_polytopes < 0 || d->reserved2 != 0)
    return RBP_E_INVALID;
  if (d->n_obstacles > 0 && (!d->box_lo || !d->box_hi)) return RBP_E_INVALID;
  if (d->n_polytopes > 0 && (!d->pob_off || !d->pob_A || !d->pob_b)) return RBP_E_INVALID;
  if (d->degree < 1 || d->degree > RBP_MAX_DEGREE) return RBP_E_SHAPE;
  const int64_t n_obst = int64_t(d->n_obstacles) + d->n_polytopes;
  const int64_t pairs = int64_t(d->n_edges) * n_obst;
  if (pairs > RBP_CUT_MAX_PAIRS || n_obst > INT32_MAX) return RBP_E_SHAPE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RBP_E_DEVICE;
  // polytope obstacles: rows to the host, vertex enumeration, checks
  std::vector<int32_t> poff, vo(size_t(d->n_polytopes) + 1, 0);
  std::vector<double> pA, pb, verts;
  int rc = RBP_OK;
  if (d->n_polytopes > 0) {
    if ((rc = d2h(poff, d->pob_off, size_t(d->n_polytopes) + 1, stream))) return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return RBP_E_DEVICE;
    if (poff[0] != 0) return RBP_E_SHAPE;
    for (int j = 0; j < d->n_polytopes; ++j) {
      const int m = poff[j + 1] - poff[j];
      if (m < 4 || m > RBP_CUT_MAX_POLY_ROWS) return RBP_E_SHAPE;
    }
    const size_t rows = size_t(poff[d->n_polytopes]);
    if ((rc = d2h(pA, d->pob_A, 3 * rows, stream)) || (rc = d2h(pb, d->pob_b, rows, stream))) return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return RBP_E_DEVICE;
    for (size_t r = 0; r < rows; ++r) {
      const double nn = pA[3 * r] * pA[3 * r] + pA[3 * r + 1] * pA[3 * r + 1] + pA[3 * r + 2] * pA[3 * r + 2];
      if (!(nn > 0.0) || !std::isfinite(nn) || !std::isfinite(pb[r])) return RBP_E_SHAPE;
    }
    for (int j = 0; j < d->n_polytopes; ++j) {
      const int r0 = poff[j], m = poff[j + 1] - r0;
      if (!polytope_bounded(pA.data() + 3 * r0, m)) return RBP_E_SHAPE;
      const size_t first = verts.size();
      const int nv = polytope_vertices(pA.data() + 3 * r0, pb.data() + r0, m, RBP_CUT_MAX_POLY_VERTS, verts);
      if (nv < 4) return RBP_E_SHAPE;   // empty, flat or too many vertices
      // full-dimensional: some four vertices span a tetrahedron
      const double* V = verts.data() + first;
      double ext = 0.0, vol = 0.0;
      for (int q = 0; q < 3 * nv; ++q) ext = std::max(ext, std::fabs(V[q] - V[q % 3]));
      for (int a = 1; a < nv && !(vol > 1e-9 * ext * ext * ext); ++a)
        for (int bq = a + 1; bq < nv; ++bq)
          for (int cq = bq + 1; cq < nv; ++cq) {
            double u[3], w[3], z[3];
            for (int k = 0; k < 3; ++k) { u[k] = V[3 * a + k] - V[k]; w[k] = V[3 * bq + k] - V[k]; z[k] = V[3 * cq + k] - V[k]; }
            const double det = u[0] * (w[1] * z[2] - w[2] * z[1]) - u[1] * (w[0] * z[2] - w[2] * z[0]) +
                               u[2] * (w[0] * z[1] - w[1] * z[0]);
            vol = std::max(vol, std::fabs(det));
          }
      if (!(vol > 1e-9 * ext * ext * ext)) return RBP_E_SHAPE;
      vo[size_t(j) + 1] = vo[size_t(j)] + nv;
    }
  }
  auto* c = new (std::nothrow) rbp_cut();
  if (!c) return RBP_E_ALLOC;
  c->device = dev;
  c->desc = *d;
  c->cap = std::max<int64_t>(pairs, 1);
  if ((rc = dalloc(&c->counter, 1)) || (rc = dalloc(&c->list, size_t(c->cap))) ||
      (rc = dalloc(&c->pv_off, vo.size())) || (rc = dalloc(&c->pv, std::max<size_t>(verts.size(), 3)))) {
    free_cut(c);
    return rc;
  }
  // the count reads 0 until the first run (which zeroes it with a kernel)
  if (hipMemsetAsync(c->counter, 0, sizeof(unsigned long long), stream) != hipSuccess ||
      hipMemcpyAsync(c->pv_off, vo.data(), vo.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream) ||
      (!verts.empty() &&
       hipMemcpyAsync(c->pv, verts.data(), verts.size() * sizeof(double), hipMemcpyHostToDevice, stream)) ||
      hipStreamSynchronize(stream) != hipSuccess) {
    free_cut(c);
    return RBP_E_DEVICE;
  }
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) n_cu = 1;
  c->qp_blocks = 4 * n_cu;   // grid-stride over the undecided pairs
  c->last_stream = stream;
  *out = c;
  return RBP_OK;
}

int rbp_cut_run(rbp_cut* c, const double* P, uint8_t* code, uint8_t* step, double* qp_dist2, int32_t* n_collide,
                hipStream_t stream) {
  if (!c) return RBP_E_INVALID;
  const rbp_cut_desc& d = c->desc;
  if (d.n_edges == 0) return RBP_OK;
  const int n_obst = d.n_obstacles + d.n_polytopes;
  if (!P || !n_collide || (n_obst > 0 && !code)) return RBP_E_INVALID;
  rbp::CutArgs a{};
  a.n_edges = d.n_edges; a.n_obst = n_obst; a.n_box = d.n_obstacles; a.degree = d.degree;
  a.P = P; a.box_lo = d.box_lo; a.box_hi = d.box_hi;
  a.pob_off = d.pob_off; a.pob_A = d.pob_A; a.pob_b = d.pob_b; a.pv_off = c->pv_off; a.pv = c->pv;
  a.code = code; a.step = step; a.qp_dist2 = qp_dist2; a.n_collide = n_collide;
  a.counter = c->counter; a.list = c->list; a.list_cap = c->cap;
  if (rbp::launch_cut(a, stream, c->qp_blocks) != hipSuccess) return RBP_E_DEVICE;
  c->last_stream = stream;
  return RBP_OK;
}

int rbp_cut_qp_count(rbp_cut* c, int64_t* n_qp) {
  if (!c || !n_qp) return RBP_E_INVALID;
  unsigned long long v = 0;
  if (hipStreamSynchronize(c->last_stream) != hipSuccess ||
      hipMemcpy(&v, c->counter, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
    return RBP_E_DEVICE;
  *n_qp = int64_t(v);
  return RBP_OK;
}

void rbp_destroy_cut(rbp_cut* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->last_stream) (void)hipStreamSynchronize(c->last_stream);
  free_cut(c);
}

struct rbp_graph {
  int device = 0;
  rbp_graph_desc desc{};
  double* A = nullptr;
  double* B = nullptr;
  double* Amin = nullptr;
  double* Bmin = nullptr;
  hipStream_t last_stream = nullptr;
};

namespace {
void free_graph(rbp_graph* g) {
  for (void* p : {static_cast<void*>(g->A), static_cast<void*>(g->B), static_cast<void*>(g->Amin),
                  static_cast<void*>(g->Bmin)})
    if (p) (void)hipFree(p);
  delete g;
}
}  // namespace

int rbp_build_graph(const rbp_graph_desc* d, hipStream_t stream, rbp_graph** out) {
  if (!d || !out) return RBP_E_INVALID;
  *out = nullptr;
  if (d->reserved != 0 || !d->F1 || !d->F2 || !d->G) return RBP_E_INVALID;
  if (d->n_nodes < 0 || d->n_nodes > RBP_GRAPH_MAX_NODES || d->dim < 1 || d->dim > RBP_GRAPH_MAX_DIM ||
      d->n_rows < 1 || d->n_rows > RBP_GRAPH_MAX_ROWS)
    return RBP_E_SHAPE;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RBP_E_DEVICE;
  auto* g = new (std::nothrow) rbp_graph();
  if (!g) return RBP_E_ALLOC;
  g->device = dev;
  g->desc = *d;
  const size_t nm = size_t(d->n_nodes) * size_t(d->n_rows);
  const size_t tm = size_t((d->n_nodes + 63) / 64) * size_t(d->n_rows);
  int rc;
  if ((rc = dalloc(&g->A, nm)) || (rc = dalloc(&g->B, nm)) || (rc = dalloc(&g->Amin, tm)) ||
      (rc = dalloc(&g->Bmin, tm))) {
    free_graph(g);
    return rc;
  }
  g->last_stream = stream;
  *out = g;
  return RBP_OK;
}

int rbp_graph_run(rbp_graph* g, const double* V, uint32_t* adj, int32_t* degree, hipStream_t stream) {
  if (!g) return RBP_E_INVALID;
  const rbp_graph_desc& d = g->desc;
  if (d.n_nodes == 0) return RBP_OK;
  if (!V || !adj || !degree) return RBP_E_INVALID;
  rbp::GraphArgs a{};
  a.n_nodes = d.n_nodes; a.dim = d.dim; a.m = d.n_rows;
  a.V = V; a.F1 = d.F1; a.F2 = d.F2; a.G = d.G;
  a.A = g->A; a.B = g->B; a.Amin = g->Amin; a.Bmin = g->Bmin;
  a.adj = adj; a.degree = degree;
  if (rbp::launch_graph(a, stream) != hipSuccess) return RBP_E_DEVICE;
  g->last_stream = stream;
  return RBP_OK;
}

void rbp_destroy_graph(rbp_graph* g) {
  if (!g) return;
  (void)hipSetDevice(g->device);
  if (g->last_stream) (void)hipStreamSynchronize(g->last_stream);
  free_graph(g);
}

static_assert(RBP_GRAPH_NOALLOC_DOUBLES == rbp::kGraphScratchDoubles, "workspace size in rbp.h");

int rbp_graph_run_noalloc(const rbp_graph_desc* d, const double* V, uint32_t* adj, int32_t* degree,
                          hipStream_t stream) {
  // every check before the first HIP call
  if (!d) return RBP_E_INVALID;
  if (d->reserved != 0 || !d->F1 || !d->F2 || !d->G) return RBP_E_INVALID;
  if (d->n_nodes < 0 || d->n_nodes > RBP_GRAPH_MAX_NODES || d->dim < 1 || d->dim > RBP_GRAPH_MAX_DIM ||
      d->n_rows < 1 || d->n_rows > RBP_GRAPH_MAX_ROWS)
    return RBP_E_SHAPE;
  const int64_t nm = int64_t(d->n_nodes) * d->n_rows;
  const int64_t tm = int64_t((d->n_nodes + 63) / 64) * d->n_rows;
  if (2 * nm + 2 * tm > rbp::kGraphScratchDoubles) return RBP_E_SCRATCH;
  if (d->n_nodes == 0) return RBP_OK;
  if (!V || !adj || !degree) return RBP_E_INVALID;
  double* ws = nullptr;
  if (rbp::graph_scratch(&ws) != hipSuccess) return RBP_E_DEVICE;
  rbp::GraphArgs a{};
  a.n_nodes = d->n_nodes; a.dim = d->dim; a.m = d->n_rows;
  a.V = V; a.F1 = d->F1; a.F2 = d->F2; a.G = d->G;
  a.A = ws; a.B = ws + nm; a.Amin = ws + 2 * nm; a.Bmin = ws + 2 * nm + tm;
  a.adj = adj; a.degree = degree;
  return rbp::launch_graph(a, stream) == hipSuccess ? RBP_OK : RBP_E_DEVICE;
}

int rbp_adjacent_hyperplanes(int32_t n, const double* X, int32_t n_obst, const double* lo, const double* hi,
                             int32_t* idx, double* point, double* plane, hipStream_t stream) {
  if (n < 0 || n_obst < 0) return RBP_E_INVALID;
  if (n == 0) return RBP_OK;
  if (!X || !idx || !point || !plane || (n_obst > 0 && (!lo || !hi))) return RBP_E_INVALID;
  return rbp::launch_hyperplanes(n, X, n_obst, lo, hi, idx, point, plane, stream) == hipSuccess ? RBP_OK
                                                                                                 : RBP_E_DEVICE;
}

struct rbp_mpc {
  int device = 0;
  rbp_mpc_desc desc{};
  double* params = nullptr;
  double ulo[3] = {0, 0, 0}, uhi[3] = {0, 0, 0};
  int ubox_ok = 0;
  hipStream_t last_stream = nullptr;
};

namespace {
// Host preparation of the MPC constants (layout of rbp::mpc_param_layout).
// State x = (p, v), z = (x, u); A = [[I, dt I], [0, I]], B = [[dt^2/2 I], [dt I]].
int mpc_params(const rbp_mpc_desc& d, const std::vector<double>& F1, const std::vector<double>& F2,
               const std::vector<double>& G, std::vector<double>& out) {
  const int m = d.n_reach;
  const double dt = d.dt, h2 = 0.5 * dt * dt;
  const rbp::MpcLayout L = rbp::mpc_param_layout(m);
  out.assign(size_t(L.total), 0.0);
  // A, B as dense 6 x 6 and 6 x 3
  double A[36] = {0}, B[18] = {0};
  for (int c = 0; c < 6; ++c) A[7 * c] = 1.0;
  for (int c = 0; c < 3; ++c) { A[6 * c + 3 + c] = dt; B[3 * c + c] = h2; B[3 * (3 + c) + c] = dt; }
  // stage Hessians: 2 blkdiag(Q, R) + 2 w J'J with J z = p_{k+1} - p_k = dt v + dt^2/2 u
  double J[27] = {0};
  for (int c = 0; c < 3; ++c) { J[9 * c + 3 + c] = dt; J[9 * c + 6 + c] = h2; }
  for (int a = 0; a < 9; ++a)
    for (int b = 0; b < 9; ++b) {
      double jj = 0.0;
      for (int c = 0; c < 3; ++c) jj += J[9 * c + a] * J[9 * c + b];
      double h0 = 2.0 * d.w_length * jj;
      if (a >= 6 && b >= 6) h0 += 2.0 * d.R[3 * (a - 6) + (b - 6)];
      double h1 = h0;
      if (a < 6 && b < 6) h1 += 2.0 * d.Q[6 * a + b];
      out[size_t(L.H0 + 9 * a + b)] = h0;
      out[size_t(L.H1 + 9 * a + b)] = h1;
    }
  for (int e = 0; e < 36; ++e) out[size_t(L.Qm + e)] = d.Q[e];
  // reachable rows in stage form: [F1 + F2 A, F2 B], scaled to unit norm
  for (int i = 0; i < m; ++i) {
    double row[9];
    for (int a = 0; a < 6; ++a) {
      double v = F1[size_t(6 * i + a)];
      for (int c = 0; c < 6; ++c) v += F2[size_t(6 * i + c)] * A[6 * c + a];
      row[a] = v;
    }
    for (int a = 0; a < 3; ++a) {
      double v = 0.0;
      for (int c = 0; c < 6; ++c) v += F2[size_t(6 * i + c)] * B[3 * c + a];
      row[6 + a] = v;
    }
    double nn = 0.0;
    for (double v : row) nn += v * v;
    nn = std::sqrt(nn);
    if (!(nn > 0.0) || !std::isfinite(nn) || !std::isfinite(G[size_t(i)])) return RBP_E_SHAPE;
    for (int a = 0; a < 9; ++a) out[size_t(L.Cr + a * L.cs + i)] = row[a] / nn;
    out[size_t(L.dr + i)] = G[size_t(i)] / nn;
  }
  // [AB B]^-1 per axis: (1/dt^3) [[dt, -dt^2/2], [-dt, 3 dt^2/2]];
  // rows (u_{N-2}, u_{N-1}), columns (target position, target velocity)
  double Mi[36] = {0};
  for (int c = 0; c < 3; ++c) {
    Mi[6 * c + c] = 1.0 / (dt * dt);
    Mi[6 * c + 3 + c] = -0.5 / dt;
    Mi[6 * (3 + c) + c] = -1.0 / (dt * dt);
    Mi[6 * (3 + c) + 3 + c] = 1.5 / dt;
  }
  for (int e = 0; e < 36; ++e) out[size_t(L.Mi + e)] = Mi[e];
  // A^2 and the eliminated last stages for a zero terminal target:
  // u_{N-2} = -L1 A^2 x, u_{N-1} = -L2 A^2 x (L1, L2: rows of Mi)
  double A2[36] = {0};
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b)
      for (int c = 0; c < 6; ++c) A2[6 * a + b] += A[6 * a + c] * A[6 * c + b];
  double U1[18], U2[18];   // u_{N-2} = U1 x, u_{N-1} = U2 x (3 x 6)
  for (int i = 0; i < 3; ++i)
    for (int b = 0; b < 6; ++b) {
      double v1 = 0.0, v2 = 0.0;
      for (int c = 0; c < 6; ++c) { v1 += Mi[6 * i + c] * A2[6 * c + b]; v2 += Mi[6 * (3 + i) + c] * A2[6 * c + b]; }
      U1[6 * i + b] = -v1;
      U2[6 * i + b] = -v2;
    }
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b) {
      out[size_t(L.T2 + 6 * a + b)] = a == b ? 1.0 : 0.0;
      double v = A[6 * a + b];     // x_{N-1} = (A + B U1) x
      for (int i = 0; i < 3; ++i) v += B[3 * a + i] * U1[6 * i + b];
      out[size_t(L.T1 + 6 * a + b)] = v;
    }
  for (int i = 0; i < 3; ++i)
    for (int b = 0; b < 6; ++b) {
      out[size_t(L.T2 + 6 * (6 + i) + b)] = U1[6 * i + b];
      out[size_t(L.T1 + 6 * (6 + i) + b)] = U2[6 * i + b];
    }
  // keep-out rows: P_j = p + a_j v + b_j u; factors (1, a_j, b_j) / |(1, a_j, b_j)|
  const double ab[4][2] = {{0.0, 0.0}, {dt / 3.0, 0.0}, {2.0 * dt / 3.0, dt * dt / 6.0}, {dt, h2}};
  for (int j = 0; j < 4; ++j) {
    const double inv = 1.0 / std::sqrt(1.0 + ab[j][0] * ab[j][0] + ab[j][1] * ab[j][1]);
    out[size_t(L.pf + 3 * j)] = inv;
    out[size_t(L.pf + 3 * j + 1)] = ab[j][0] * inv;
    out[size_t(L.pf + 3 * j + 2)] = ab[j][1] * inv;
  }
  return RBP_OK;
}

// Box of every input u_k allowed by the reachable rows that act on the input
// alone: rows of F1 x_k + F2 x_{k+1} <= G whose coefficients on x_k vanish
// exactly once x_{k+1} = A x_k + B u_k is substituted, g'u <= G_i with
// g = (F2 B)_i.  Bound propagation over the three components from an
// unbounded start (each row bounds one component given the bounds of the
// others); the result is widened by 1e-12 (1 + |bound|) against rounding.
// Returns false when a component stays unbounded.
bool mpc_input_box(int m, double dt, const std::vector<double>& F1, const std::vector<double>& F2,
                   const std::vector<double>& G, double lo[3], double hi[3]) {
  const double h2 = 0.5 * dt * dt;
  std::vector<std::array<double, 3>> gs;
  std::vector<double> ds;
  for (int i = 0; i < m; ++i) {
    bool input_only = true;
    for (int a = 0; a < 6 && input_only; ++a) {
      // (F1 + F2 A) column a; A = [[I, dt I], [0, I]]
      double v = F1[size_t(6 * i + a)] + F2[size_t(6 * i + a)];
      if (a >= 3) v += dt * F2[size_t(6 * i + a - 3)];
      input_only = v == 0.0;
    }
    if (!input_only) continue;
    std::array<double, 3> g{};
    for (int c = 0; c < 3; ++c) g[c] = h2 * F2[size_t(6 * i + c)] + dt * F2[size_t(6 * i + 3 + c)];
    gs.push_back(g);
    ds.push_back(G[size_t(i)]);
  }
  const double inf = std::numeric_limits<double>::infinity();
  for (int c = 0; c < 3; ++c) { lo[c] = -inf; hi[c] = inf; }
  for (int sweep = 0; sweep < 8; ++sweep)
    for (size_t r = 0; r < gs.size(); ++r)
      for (int c = 0; c < 3; ++c) {
        const double gc = gs[r][c];
        if (gc == 0.0) continue;
        double rest = 0.0;   // min of the other terms
        for (int c2 = 0; c2 < 3; ++c2) {
          if (c2 == c || gs[r][c2] == 0.0) continue;
          rest += gs[r][c2] > 0.0 ? gs[r][c2] * lo[c2] : gs[r][c2] * hi[c2];
        }
        if (!std::isfinite(rest)) continue;
        const double b = (ds[r] - rest) / gc;
        if (gc > 0.0) hi[c] = std::min(hi[c], b);
        else lo[c] = std::max(lo[c], b);
      }
  for (int c = 0; c < 3; ++c) {
    if (!std::isfinite(lo[c]) || !std::isfinite(hi[c]) || lo[c] > hi[c]) return false;
    lo[c] -= 1e-12 * (1.0 + std::fabs(lo[c]));
    hi[c] += 1e-12 * (1.0 + std::fabs(hi[c]));
  }
  return true;
}

bool sym_psd_diag(const double* M, int n) {
  for (int a = 0; a < n; ++a) {
    if (!std::isfinite(M[n * a + a]) || M[n * a + a] < 0.0) return false;
    for (int b = 0; b < n; ++b)
      if (!std::isfinite(M[n * a + b]) || std::fabs(M[n * a + b] - M[n * b + a]) > 1e-12 * (1.0 + std::fabs(M[n * a + b])))
        return false;
  }
  return true;
}

bool spd3(const double* R) {
  if (!sym_psd_diag(R, 3)) return false;
  const double l00 = R[0];
  if (!(l00 > 0.0)) return false;
  const double a = std::sqrt(l00), l10 = R[3] / a, l20 = R[6] / a;
  const double d1 = R[4] - l10 * l10;
  if (!(d1 > 0.0)) return false;
  const double b = std::sqrt(d1), l21 = (R[7] - l20 * l10) / b;
  return R[8] - l20 * l20 - l21 * l21 > 0.0;
}
}  // namespace

int rbp_build_mpc(const rbp_mpc_desc* d, hipStream_t stream, rbp_mpc** out) {
  if (!d || !out) return RBP_E_INVALID;
  *out = nullptr;
  if (d->reserved != 0 || !(d->dt > 0.0) || !std::isfinite(d->dt) || !(d->w_length >= 0.0) ||
      !std::isfinite(d->w_length) || !sym_psd_diag(d->Q, 6) || !spd3(d->R))
    return RBP_E_INVALID;
  if (d->n_instances < 0 || d->horizon < 2 || d->horizon > RBP_MPC_MAX_HORIZON || d->n_reach < 0 ||
      d->n_reach > RBP_MPC_MAX_REACH)
    return RBP_E_SHAPE;
  const int m = d->n_reach;
  if (m > 0 && (!d->F1 || !d->F2 || !d->G)) return RBP_E_INVALID;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RBP_E_DEVICE;
  std::vector<double> F1, F2, G, prm;
  int rc;
  if (m > 0) {
    if ((rc = d2h(F1, d->F1, size_t(6 * m), stream)) || (rc = d2h(F2, d->F2, size_t(6 * m), stream)) ||
        (rc = d2h(G, d->G, size_t(m), stream)))
      return rc;
    if (hipStreamSynchronize(stream) != hipSuccess) return RBP_E_DEVICE;
  }
  if ((rc = mpc_params(*d, F1, F2, G, prm))) return rc;
  auto* q = new (std::nothrow) rbp_mpc();
  if (!q) return RBP_E_ALLOC;
  q->device = dev;
  q->desc = *d;
  q->ubox_ok = mpc_input_box(m, d->dt, F1, F2, G, q->ulo, q->uhi) ? 1 : 0;
  if ((rc = dalloc(&q->params, prm.size()))) { delete q; return rc; }
  if (hipMemcpyAsync(q->params, prm.data(), prm.size() * sizeof(double), hipMemcpyHostToDevice, stream) ||
      hipStreamSynchronize(stream)) {
    (void)hipFree(q->params);
    delete q;
    return RBP_E_DEVICE;
  }
  q->last_stream = stream;
  *out = q;
  return RBP_OK;
}

int rbp_mpc_solve(rbp_mpc* q, const double* x0, const double* ref, const double* planes, int32_t max_iters,
                  double tol, double* X, double* U, double* cost, int32_t* status, double* kkt, int32_t* iters,
                  hipStream_t stream) {
  if (!q || max_iters <= 0 || !(tol > 0.0)) return RBP_E_INVALID;
  const rbp_mpc_desc& d = q->desc;
  if (d.n_instances == 0) return RBP_OK;
  if (!x0 || !ref || !planes || !X || !U || !cost || !status || !kkt) return RBP_E_INVALID;
  rbp::MpcArgs a{};
  a.n = d.n_instances; a.N = d.horizon; a.m = d.n_reach;
  a.max_iters = max_iters; a.tol = tol; a.dt = d.dt;
  a.params = q->params;
  a.x0 = x0; a.ref = ref; a.planes = planes;
  a.X = X; a.U = U; a.cost = cost; a.status = status; a.kkt = kkt; a.iters = iters;
  for (int c = 0; c < 3; ++c) { a.ulo[c] = q->ulo[c]; a.uhi[c] = q->uhi[c]; }
  a.ubox_ok = q->ubox_ok;
  if (rbp::launch_mpc(a, stream) != hipSuccess) return RBP_E_DEVICE;
  q->last_stream = stream;
  return RBP_OK;
}

void rbp_destroy_mpc(rbp_mpc* q) {
  if (!q) return;
  (void)hipSetDevice(q->device);
  if (q->last_stream) (void)hipStreamSynchronize(q->last_stream);
  if (q->params) (void)hipFree(q->params);
  delete q;
}

}  // extern "C"
