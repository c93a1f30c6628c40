// Internal interface between the C ABI (rbp_api.cpp) and the kernels
// (rbp_kernels.hip).  Not part of the public header.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "rbp_consts.hpp"

namespace rbp {

// Per-instance row numbering used by the solver, the stored active sets and
// the backward pass (p = degree, nf = faces of the instance's polytope,
// r = reachable rows):
//   faces  : id = s*nf + j           s = 0..p-2 (control point s+1), j < nf
//   vel    : id = F + 3k + c         k = 0..p-1, c = 0..2   (F = (p-1) nf)
//   acc    : id = F + 3p + 3k + c    k = 0..p-2
//   reach  : id = F + 6p - 3 + l     l < r
// Face and reachable rows are one-sided (upper bound); difference rows are
// two-sided.  An active constraint is (id, side) with side = +1 (upper) or
// -1 (lower).

struct LdsDims {
  int nmax;    // 3 (pmax - 1)
  int ncol;    // 3 (pmax + 1)
  int r_cap;   // max reachable rows
  int nf_cap;  // max faces
  int m_cap;   // max rows
  // byte offsets
  int o_Hd, o_Af, o_rowval, o_ybuf, o_vec, o_scal, o_acte, o_lam, o_actid, o_actside, o_cst, o_Rd, o_region;
  int o_Hf, o_Aff, o_vbuf, o_xb1, o_xb2, o_Kx;   // ADMM part of region
  int o_Q1, o_R, o_Ri;                            // polish part of region
  int bytes;
};

// Per-instance descriptor in work-order position, built by rbp_build_batch
// from the index arrays: one block reads its instance's offsets with a few
// uniform loads instead of a chain of dependent ones.
struct alignas(16) InstDesc {
  int32_t inst, p, f0, nf;   // instance, degree, first face of its polytope, faces
  int32_t r, pad0;           // reachable rows
  int64_t r0;                // first reachable row (h0, G)
  int64_t hb, po;            // element offset of its H block, control-point offset of P
  int64_t fo, pad1;          // offset of its faces in grad_b
};

struct SolveArgs {
  int N;                     // solve: end of the launch's range in the work order
  const int32_t* degree;
  const double* T;
  const int32_t* poly_off;
  const double* A_face;
  const double* b_face;
  const int32_t* poly_idx;
  const int64_t* reach_off;
  const int64_t* H_off;
  const int32_t* reach_idx;  // nullable: reachable block of each instance (else the instance's own)
  int pin_v0;                // 1: (p/T)(P_1 - P_0) = x0[3:6] replaces the k = 0 velocity rows
  const double* H;
  const double* h0;
  const double* G;
  double vmax, amax;
  const double* x0;
  const double* goal;
  const int64_t* pt_off;     // per-instance offset in control points (sum of p+1)
  const int32_t* order;      // work order (nullable): block b solves order[b]
  const InstDesc* desc;      // [N] descriptors in work-order position
  int inst_base;             // first work-order position of the launch (block b -> inst_base + b)
  double* P_out;
  double* cost_out;
  int32_t* status_out;
  double* kkt_out;
  int32_t* iters_out;        // nullable, 2 per instance: ADMM iterations, polish steps
  // state kept for the backward pass
  int store;
  int debug_fill;            // 1: fill the workgroup's LDS with NaN first
  int32_t* st_q;             // active count per instance
  int32_t* st_id;            // [N * nmax] row ids
  int32_t* st_side;          // [N * nmax] sides
  double* st_lam;            // [N * st_stride] multipliers
  double* st_qr;             // [N * 2 st_stride^2] final factor: q rows of Q1, then the q x q R block
  int st_stride;             // entries per instance in st_id / st_side / st_lam
  // forward results kept for the backward pass (written when store is set)
  int32_t* fw_status;        // [N]
  double* fw_nu;             // [N][6] multipliers of the pinned start and goal coordinates
  // options
  int admm_iters;
  float rho, alpha;
  int max_steps;
  double feas_tol;
  double kkt_tol;
  LdsDims dims;
};

struct BackArgs {
  int N;                     // end of the launch's range in the work order
  const int32_t* order;      // work order (nullable): block b handles order[inst_base + b]
  const InstDesc* desc;      // [N] descriptors in work-order position
  int inst_base;
  int debug_fill;            // 1: fill the workgroup's LDS with NaN first
  int st_stride;
  const int32_t* degree;
  const double* T;
  const int32_t* poly_off;
  const double* A_face;
  const int32_t* poly_idx;
  const int64_t* reach_off;
  const int64_t* H_off;
  const int32_t* reach_idx;  // nullable: reachable block of each instance (else the instance's own)
  int pin_v0;                // 1: (p/T)(P_1 - P_0) = x0[3:6] replaces the k = 0 velocity rows
  const double* H;
  const double* G;
  double vmax, amax;
  const int64_t* pt_off;
  const int64_t* face_off;   // per-instance offset of its faces in grad_b
  const double* nu;          // [N][6] multipliers of the pinned coordinates (forward pass)
  const int32_t* status;
  const int32_t* st_q;
  const int32_t* st_id;
  const int32_t* st_side;
  const double* st_lam;
  const double* st_qr;
  const double* grad_P;      // nullable
  const double* grad_cost;   // nullable
  double* grad_x0;
  double* grad_goal;
  double* grad_b;
  int32_t* flags;            // nullable: 1 when the active rows are (near) dependent
  LdsDims dims;
};

// ---- multi-segment paths (rbp_chain.hip)
struct ChainDims {
  int s_cap, nf_cap, r_cap, q_cap, nf_pts_cap, ng_cap, n_cap, m_cap;
  int o_segi, o_seg64, o_Af, o_bfs, o_fan, o_rb, o_rn, o_Pseg, o_gfull, o_G1b, o_L1b, o_L1r, o_qv, o_x, o_scal,
      o_cand, o_bits;
  int o_Kb, o_zr, o_yr, o_accp, o_Pf, o_xt, o_Cs, o_Wm;          // ADMM part of the region
  int o_LS, o_LSd, o_beta, o_acte, o_u, o_cvec, o_actid;          // polish part of the region
  int bytes;
};

struct ChainArgs {
  int N;
  int P;
  double T, vmax, amax;
  const int64_t* seg_off;
  const int32_t* poly_off;
  const double* A_face;
  const double* b_face;
  const int32_t* poly_idx;
  const int64_t* reach_off;
  const int64_t* H_off;
  const double* H;
  const double* h0;
  const double* G;
  const double* x0;
  const double* goal;
  const int32_t* order;      // work order: block b solves order[inst_base + b]
  int inst_base;             // N is the end of the launch's range
  double* P_out;
  double* cost_out;
  int32_t* status_out;
  double* kkt_out;
  int32_t* iters_out;
  int admm_iters;
  float rho, alpha;
  int max_steps;
  double feas_tol, kkt_tol;
  ChainDims dims;
  int q_full;       // working-set cap of the full pass; a smaller dims.q_cap marks overflows for retry
  int retry_only;   // solve only the paths a reduced-cap pass marked for retry
  // working set of a path at its overflow (written by the reduced-cap pass,
  // read by the full pass, which continues from it): row keys 2 id + (side > 0)
  int32_t* ws_keys;  // [N][ws_stride]
  int32_t* ws_meta;  // [N][2]: rows, polish steps taken
  int ws_stride;
};

// ---- cutting graph edges against box obstacles (rbp_cut.hip)
struct CutArgs {
  int n_edges, n_obst, degree;
  int n_box;                 // obstacles 0 .. n_box-1 are boxes, the rest polytopes
  const double* P;           // [n_edges][degree+1][3]
  const double* box_lo;      // [n_box][3]
  const double* box_hi;      // [n_box][3]
  const int32_t* pob_off;    // [n_obst - n_box + 1] row offsets of the polytopes
  const double* pob_A;       // [rows][3]
  const double* pob_b;       // [rows]
  const int32_t* pv_off;     // [n_obst - n_box + 1] vertex offsets
  const double* pv;          // [vertices][3]
  uint8_t* code;             // [n_obst][n_edges]: 1 free, 0 may collide
  uint8_t* step;             // nullable [n_obst][n_edges]: 1, 2 or 3 (Alg. 2 step that decided)
  double* qp_dist2;          // nullable [n_obst][n_edges]: |delta*|^2 where step 3 ran, NaN elsewhere
  int32_t* n_collide;        // [n_edges]: obstacles the edge may collide with
  unsigned long long* counter;   // pairs appended to the list (device scalar)
  int64_t* list;             // undecided pairs (o << 32 | e)
  int64_t list_cap;
};
hipError_t launch_cut(const CutArgs& a, hipStream_t s, int qp_blocks);

// ---- building the graph and adjacent hyperplanes (rbp_graph.hip)
struct GraphArgs {
  int n_nodes, dim, m;
  const double* V;           // [n_nodes][dim]
  const double* F1;          // [m][dim] columns of F on the start node
  const double* F2;          // [m][dim] columns of F on the end node
  const double* G;           // [m]
  double* A;                 // [n_nodes][m] F1 v (workspace)
  double* B;                 // [n_nodes][m] F2 v - G (workspace)
  double* Amin;              // [n_tiles][m] tile minima (workspace)
  double* Bmin;
  uint32_t* adj;             // [n_nodes][ceil(n_nodes / 32)] bitmask
  int32_t* degree;           // [n_nodes]
};
hipError_t launch_graph(const GraphArgs& a, hipStream_t s);
// Fixed device workspace of rbp_graph_run_noalloc, in doubles (8 MiB).
constexpr int64_t kGraphScratchDoubles = int64_t(1) << 20;
// Device address of the current GPU's copy of that workspace (looked up once
// per device with hipGetSymbolAddress, then cached).
hipError_t graph_scratch(double** out);
hipError_t launch_hyperplanes(int n, const double* X, int n_obst, const double* lo, const double* hi, int32_t* idx,
                              double* point, double* plane, hipStream_t s);

// Batched MPC refinement (one wave per instance).  params: constants built
// on the host by the library (layout in mpc_param_layout).
struct MpcLayout {
  int H1, H0, Qm, Cr, dr, T2, T1, Mi, pf, total;   // offsets in doubles
  int cs;                                          // column stride of Cr (odd)
};
__host__ __device__ inline MpcLayout mpc_param_layout(int m) {
  MpcLayout L{};
  int o = 0;
  L.H1 = o; o += 81;      // stage Hessian, k >= 1 (9 x 9, z = [x; u])
  L.H0 = o; o += 81;      // stage Hessian, k = 0 (no tracking)
  L.Qm = o; o += 36;      // tracking weight Q
  L.cs = m | 1;
  L.Cr = o; o += 9 * L.cs;  // reachable rows in stage form, unit norm, stored by
                            // column: entry (i, a) at a * cs + i (odd stride)
  L.dr = o; o += m;       // their right-hand sides
  L.T2 = o; o += 54;      // z_{N-2} = T2 x_{N-2}   (last two stages eliminated)
  L.T1 = o; o += 54;      // z_{N-1} = T1 x_{N-2}
  L.Mi = o; o += 36;      // [AB B]^-1 (start point: terminal inputs)
  L.pf = o; o += 12;      // plane-row factors (1, a_j, b_j) / |(1, a_j, b_j)|
  L.total = o;
  return L;
}
struct MpcArgs {
  int n;                     // instances
  int N, m;                  // horizon, reachable rows per step
  int max_iters;
  double tol;                // complementarity / residual target
  double dt;
  const double* params;      // [mpc_param_layout(m).total]
  const double* x0;          // [n][6]
  const double* ref;         // [n][N+1][6]
  const double* planes;      // [n][N][4]
  double* X;                 // [n][N+1][6]
  double* U;                 // [n][N][3]
  double* cost;              // [n]
  int32_t* status;           // [n]
  double* kkt;               // [n]
  int32_t* iters;            // [n] or null
  // box of every input u_k from the rows that act on the input alone
  // (ubox_ok = 0: those rows leave some component unbounded, no certificate)
  double ulo[3], uhi[3];
  int ubox_ok;
};
size_t mpc_lds_bytes(int N, int m);
hipError_t launch_mpc(const MpcArgs& a, hipStream_t s);

// admm = false: no room for the ADMM iteration (polish only)
LdsDims make_dims(int pmax, int r_cap, int nf_cap, int real_bytes, bool admm);
// LDS of the backward pass alone (its own, smaller carve: more waves resident)
LdsDims make_back_dims(int pmax, int nf_cap);
ChainDims make_chain_dims(int p, int s_cap, int nf_cap, int r_cap, int q_cap, bool admm);
hipError_t upload_chain_constants(int device);
hipError_t launch_chains(const ChainArgs& a, hipStream_t s);
hipError_t upload_constants(int device);
// launch shapes of the grouped solve: waves (instances) per workgroup and the
// waves per SIMD the register budget is sized for
constexpr int kShapeW1E2 = 0, kShapeW1E1 = 1, kShapeW2E2 = 2;
constexpr int kShapeWaves[3] = {1, 1, 2};
// default shape (rbp_kernels.hip)
hipError_t launch_solve(const SolveArgs& a, int n_blocks, hipStream_t s, bool fp64_iters, int pfix);
hipError_t launch_backward(const BackArgs& a, int n_blocks, hipStream_t s, int pfix);
// other shapes and the single-launch schedule (rbp_kernels_var.hip, FP32
// iterations or polish only); that unit has its own constant table
hipError_t upload_constants_var(int device);
hipError_t launch_solve_shape(const SolveArgs& a, int n_inst, hipStream_t s, int pfix, int shape);
hipError_t launch_solve_all(const SolveArgs& a, int n_inst, hipStream_t s);
hipError_t launch_backward_all(const BackArgs& a, int n_inst, hipStream_t s);

}  // namespace rbp
