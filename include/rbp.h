/*
 * rbp.h -- batched reachable-Bezier-polytope segment QPs on AMD MI355X (gfx950).
 *
 * One instance is one candidate graph edge of the Bezier-graph planner
 * (Csomay-Shanklin, Compton, Ames, "Dynamically Feasible Path Planning in
 * Cluttered Environments via Reachable Bezier Polytopes", Sec. II-B and III):
 * a degree-p Bezier curve on [0, T] in R^3, control points P_0..P_p,
 *
 *   minimise    int_0^T |b''(t)|^2 dt        (closed-form Bernstein Hessian)
 *   subject to  A_f P_k <= b_f          for every control point k
 *                                        (free-space polytope; by the
 *                                        convex-hull property, Property 1,
 *                                        the whole curve stays inside)
 *               |p/T (P_{k+1} - P_k)|      <= vmax   componentwise
 *               |p(p-1)/T^2 Delta^2 P_k|   <= amax   componentwise
 *               H vec(P) <= h0 + G x0        (reachable Bezier polytope,
 *                                             Theorem 2, affine in x0)
 *               P_0 = x0[0:3],  P_p = goal   (the edge joins two waypoints)
 *               [optional] (p/T)(P_1 - P_0) = x0[3:6]  (pinned start velocity)
 *
 * vec(P) is point-major: element 3k + c is coordinate c of control point k.
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers (hipMalloc'd memory or torch
 *     tensors on the GPU), row-major and contiguous, unless stated otherwise.
 *   - Calls are enqueued on the given HIP stream and are asynchronous with
 *     respect to the host, except rbp_build_batch, which copies the index
 *     arrays to the host to validate them and synchronises the stream.
 *   - The caller owns every buffer it passes.  A batch owns its internal
 *     state (packed offsets, work order, stored forward state) until
 *     rbp_destroy_batch.  The problem arrays named in rbp_problem_desc are
 *     read, not copied: they must stay valid and unchanged while the batch
 *     is used.
 *   - A batch is not re-entrant: do not run two calls on one batch
 *     concurrently on different streams.
 *   - Grouped launches (batches of several degrees or row classes, path
 *     batches of several lengths) run their groups on the caller's stream and
 *     on three side streams of the device, made at the first batch built on
 *     it and shared by every batch until the process ends; the side streams
 *     are forked from the caller's stream and joined back into it with
 *     events, so every call stays ordered on the caller's stream (and can be
 *     captured in a graph there).  Calls on different caller streams share
 *     the side streams and may wait for each other.
 *   - Return value: RBP_OK (0) or a negative RBP_E_* code; nothing throws
 *     across this interface.  Per-instance outcomes are reported in
 *     status_out (RBP_SOLVED ... RBP_INVALID_INPUT).
 */
#ifndef RBP_H_
#define RBP_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* call results */
#define RBP_OK 0
#define RBP_E_INVALID (-1) /* null pointer or out-of-range scalar argument        */
#define RBP_E_SHAPE (-2)   /* inconsistent offsets, degree or size out of range    */
#define RBP_E_ALLOC (-3)   /* device allocation failed                             */
#define RBP_E_DEVICE (-4)  /* a HIP runtime call or kernel launch failed           */
#define RBP_E_STATE (-5)   /* backward without a stored forward pass               */
#define RBP_E_SCRATCH (-6) /* problem exceeds the fixed workspace of an
                              allocation-free entry point                         */

/* per-instance status */
#define RBP_SOLVED 0         /* optimum found, scaled KKT residual <= kkt_tol      */
#define RBP_INFEASIBLE 1     /* Farkas certificate verified in FP64                */
#define RBP_MAXITER 2        /* reserved                                           */
#define RBP_POLISH_FAILED 3  /* active-set polish hit its step cap, or its
                                infeasibility certificate did not verify          */
#define RBP_NUMERICAL 4      /* polished point misses the KKT tolerance            */
#define RBP_INVALID_INPUT 5  /* non-finite input, T <= 0 or a zero face normal     */

#define RBP_MIN_DEGREE 3
#define RBP_MAX_DEGREE 9
#define RBP_MAX_FACES 64     /* faces per polytope                                 */
#define RBP_MAX_REACH 128    /* reachable rows per instance                        */

/*
 * Problem description (device pointers).  N instances share a table of
 * n_poly free-space polytopes (the keep-in regions of the paper's convex
 * decomposition); instance i uses polytope poly_idx[i].
 */
typedef struct rbp_problem_desc {
  int32_t n_instances;        /* N >= 0                                          */
  int32_t n_poly;             /* polytopes in the table (>= 1 when N > 0)        */
  const int32_t* degree;      /* [N] Bezier degree p, RBP_MIN..RBP_MAX_DEGREE    */
  const double* T;            /* [N] segment duration, > 0                       */
  const int32_t* poly_off;    /* [n_poly+1] polytope j owns faces
                                 poly_off[j] .. poly_off[j+1]-1, poly_off[0] = 0,
                                 1..RBP_MAX_FACES faces each                      */
  const double* A_face;       /* [F][3] outward face normals (non-zero)          */
  const double* b_face;       /* [F] face offsets: A_face[f] . x <= b_face[f]    */
  const int32_t* poly_idx;    /* [N] polytope of each instance                   */
  const int64_t* reach_off;   /* [N+1] reachable-row offsets, reach_off[0] = 0,
                                 r_i = reach_off[i+1]-reach_off[i] in 0..128      */
  const int64_t* H_off;       /* [N+1] element offsets into H; instance i holds
                                 r_i x 3(p_i+1) doubles, row-major                */
  const double* H;            /* reachable-polytope rows over vec(P)             */
  const double* h0;           /* [R] right-hand sides, R = reach_off[N]          */
  const double* G;            /* [R][6] dependence of the right-hand side on x0  */
  double vmax;                /* velocity bound, > 0                             */
  double amax;                /* acceleration bound, > 0                         */
  /* Shared reachable polytopes (Sec. III-A: the reachable set of Theorem 2
   * depends only on the dynamics, the bounds and the duration, so one table
   * entry can serve every edge).  reach_idx == NULL: reach_off and H_off
   * above have N+1 entries, one block per instance, and n_reach is ignored.
   * reach_idx != NULL: reach_off and H_off have n_reach+1 entries indexing a
   * table of n_reach >= 1 blocks, and instance i uses block reach_idx[i]
   * (0 <= reach_idx[i] < n_reach), whose H part must have r x 3(p_i+1)
   * elements for that instance's degree.  The right-hand side h0 + G x0 is
   * still formed per instance from its own x0.  rbp_build_batch checks all
   * of this (RBP_E_SHAPE otherwise). */
  int32_t n_reach;
  const int32_t* reach_idx;   /* [N] or NULL                                     */
  /* 1: the start velocity is pinned as well as the start position (the
   * full-state start of Lemma 1): every instance also satisfies
   * (p/T)(P_1 - P_0) = x0[3:6], the derivative of the curve at t = 0.  Its
   * k = 0 velocity rows then reduce to |x0[3+c]| <= vmax, a constant test
   * (RBP_INFEASIBLE when it fails).  0: only P_0 is pinned.  Other values:
   * RBP_E_INVALID. */
  int32_t pin_start_velocity;
} rbp_problem_desc;

typedef struct rbp_solve_opts {
  int32_t admm_iters;         /* FP32 ADMM iterations before the polish (>= 0)   */
  float rho;                  /* ADMM penalty (> 0)                               */
  float alpha;                /* ADMM relaxation, in (0, 2)                       */
  int32_t max_polish_steps;   /* FP64 active-set step cap; 0 = 8 n + 64          */
  double feas_tol;            /* polish primal tolerance, relative (> 0)         */
  double kkt_tol;             /* SOLVED requires scaled KKT residual <= this     */
  int32_t store_for_backward; /* keep the active set for rbp_backward             */
  int32_t plain;              /* 1: FP64 iterations, one kernel launch per
                                 instance (the unbatched baseline)                */
  int32_t launch_shape;       /* grouped schedule: 0 = one instance (wavefront)
                                 per workgroup, registers sized for two
                                 wavefronts per SIMD; 1 = one per workgroup,
                                 registers for one wavefront per SIMD; 2 = two
                                 instances per workgroup, each wavefront on its
                                 own LDS slice.  Ignored with plain, with
                                 schedule 1, and with FP64 iterations       */
  int32_t schedule;           /* 0 = one launch per (degree, reachable-row
                                 class) group, LDS sized per group; 1 = one
                                 launch for the whole batch (degree chosen in
                                 the kernel, LDS sized for the largest
                                 instance).  The backward pass follows the
                                 schedule of the forward pass it differentiates */
  int32_t debug_fill_lds;     /* 1: every segment workgroup fills its LDS with
                                 NaN before use (forward pass and the backward
                                 pass of that forward), so a read of a value
                                 never written shows up in the outputs; 0 for
                                 normal runs.  Ignored by rbp_solve_chains    */
  int32_t reserved;           /* must be 0                                     */
} rbp_solve_opts;

/* Sizes of the variable-length outputs of a batch (host struct). */
typedef struct rbp_batch_sizes {
  int32_t n_instances;
  int32_t max_degree;
  int64_t points_total;       /* sum_i (p_i + 1): P_out holds 3 * points_total   */
  int64_t faces_total;        /* sum_i n_f(poly_idx[i]): length of grad_b        */
} rbp_batch_sizes;

typedef struct rbp_batch rbp_batch;

/* Fills *o with the defaults: admm_iters 10, rho 0.1, alpha 1.6,
 * max_polish_steps 0, feas_tol 1e-11, kkt_tol 1e-6, store_for_backward 1,
 * plain 0, launch_shape 0, schedule 0. */
void rbp_default_opts(rbp_solve_opts* o);

/*
 * Validates the description (index arrays are copied to the host; the call
 * synchronises `stream`), computes per-instance output offsets and a work
 * order, uploads the per-degree constant tables to the current device and
 * allocates the forward state kept for rbp_backward (per instance: the final
 * working set, its factor in a slot of 2 (3(pmax-1))^2 doubles, with pmax the
 * largest degree, and the multipliers of the pinned coordinates).  On success *out owns the new batch.
 * Errors: RBP_E_INVALID (null pointers, vmax/amax <= 0), RBP_E_SHAPE (offsets
 * not monotone, sizes or degrees out of range, H_off inconsistent with the
 * degrees and row counts), RBP_E_ALLOC, RBP_E_DEVICE.
 */
int rbp_build_batch(const rbp_problem_desc* desc, hipStream_t stream, rbp_batch** out);

/* Output sizes of a built batch.  Errors: RBP_E_INVALID. */
int rbp_batch_get_sizes(const rbp_batch* batch, rbp_batch_sizes* out);

/*
 * Forward pass over all instances: the segment QP above (the per-edge curve
 * of the Bezier graph of Sec. II-B, dynamically feasible by Theorem 2 and
 * collision-free by Property 1).  With opts->admm_iters > 0 an FP32 ADMM
 * stage runs first and proposes a working set; with admm_iters == 0 it is
 * skipped.  Either way the FP64 dual active-set polish decides every result:
 * the exact optimum, or infeasibility with a certificate verified in FP64 (a
 * Farkas vector, or a dual value of the polish's multipliers above every
 * objective value in the box that the velocity rows chained from both pinned
 * ends give: weak duality).
 *   x0      [N][6]   start state (position, velocity); P_0 = x0[0:3]
 *   goal    [N][3]   end waypoint; P_p = goal
 *   b_face  [F] or NULL: replaces desc->b_face for this call (and backward)
 *   opts    host pointer or NULL (defaults)
 *   P_out   [3 * points_total]: instance i at 3 * sum_{i'<i}(p_i'+1);
 *           NaN unless SOLVED
 *   cost_out   [N] optimal cost; +inf if INFEASIBLE, NaN on other failures
 *   status_out [N] RBP_SOLVED ... RBP_INVALID_INPUT
 *   kkt_out    [N] max of the scaled primal, dual and complementarity
 *              residuals of the polished point (NaN unless SOLVED/NUMERICAL)
 *   iters_out  [N][2] or NULL: ADMM iterations, polish steps
 * Errors: RBP_E_INVALID (null required pointer, bad option), RBP_E_DEVICE.
 */
int rbp_solve_batch(rbp_batch* batch, const double* x0, const double* goal, const double* b_face,
                    const rbp_solve_opts* opts, double* P_out, double* cost_out,
                    int32_t* status_out, double* kkt_out, int32_t* iters_out, hipStream_t stream);

/*
 * Vector-Jacobian product of the last forward pass (which must have run with
 * store_for_backward) for the loss  l = sum_i grad_P_i . P*_i + grad_cost_i f*_i,
 * by implicit differentiation of the KKT system on the polished active set
 * (with the QR factor of its whitened normals that the forward pass kept).
 *   grad_P    [3 * points_total] or NULL (zero)
 *   grad_cost [N] or NULL (zero)
 *   grad_x0   [N][6], grad_goal [N][3]
 *   grad_b    [faces_total]: d l / d b_face for the faces of instance i's
 *             polytope, at sum_{i'<i} n_f(i'); callers with a shared table
 *             scatter-add these into it
 *   flags_out [N] or NULL: 1 when the active rows are (nearly) linearly
 *             dependent, so the derivative is not unique
 * Instances that are not SOLVED get zero gradients.
 * Errors: RBP_E_INVALID, RBP_E_STATE (no stored forward), RBP_E_DEVICE.
 */
int rbp_backward(rbp_batch* batch, const double* grad_P, const double* grad_cost, double* grad_x0,
                 double* grad_goal, double* grad_b, int32_t* flags_out, hipStream_t stream);

/* Releases the batch and its device state (no-op for NULL).  Synchronises the
 * batch's last stream first. */
void rbp_destroy_batch(rbp_batch* batch);

/*
 * Multi-segment paths.  A path is S segments of one degree (7) and duration T
 * joined with continuous position, velocity and acceleration (equal
 * durations: C0, C1 and C2 conditions on the control points); start and goal
 * pinned.  Segment s keeps its control points in polytope poly_idx[s] and
 * satisfies its reachable rows  H_s vec(P^s) <= h0_s + G_s x0_s,  where x0_s is
 * the path's start state for the first segment and the join state
 * (P^s_0, p/T (P^s_1 - P^s_0)) for the others.  Device pointers throughout.
 */
#define RBP_CHAIN_DEGREE 7
#define RBP_CHAIN_MAX_SEGMENTS 12

typedef struct rbp_chain_desc {
  int32_t n_chains;           /* N >= 0                                          */
  int32_t n_poly;             /* polytopes in the table                          */
  int32_t degree;             /* RBP_CHAIN_DEGREE                                */
  int32_t reserved;           /* 0                                               */
  double T;                   /* segment duration, > 0                           */
  double vmax, amax;          /* > 0                                             */
  const int64_t* seg_off;     /* [N+1] path c owns segments seg_off[c]..seg_off[c+1]-1,
                                 1..RBP_CHAIN_MAX_SEGMENTS each                   */
  const int32_t* poly_off;    /* [n_poly+1] as in rbp_problem_desc               */
  const double* A_face;       /* [F][3]                                          */
  const double* b_face;       /* [F]                                             */
  const int32_t* poly_idx;    /* [n_seg] polytope of each segment                */
  const int64_t* reach_off;   /* [n_seg+1] reachable-row offsets, 0..128 rows    */
  const int64_t* H_off;       /* [n_seg+1] element offsets, r x 3(p+1) each      */
  const double* H;
  const double* h0;           /* [R]                                             */
  const double* G;            /* [R][6]                                          */
} rbp_chain_desc;

typedef struct rbp_chains rbp_chains;

/* Validates (index arrays copied to the host, stream synchronised) and builds
 * a path batch.  Errors as rbp_build_batch; degree other than 7 or more than
 * RBP_CHAIN_MAX_SEGMENTS segments is RBP_E_SHAPE. */
int rbp_build_chains(const rbp_chain_desc* desc, hipStream_t stream, rbp_chains** out);

/* points_total = sum over paths of S (p+1): P_out holds 3 points_total
 * doubles, path c at 3 (p+1) seg_off[c]; faces_total is 0. */
int rbp_chains_get_sizes(const rbp_chains* chains, rbp_batch_sizes* out);

/*
 * Forward pass over all paths: FP32 ADMM warm start (admm_iters > 0) with a
 * banded KKT matrix in LDS, FP64 dual active-set polish with banded Cholesky
 * solves.  Infeasibility is reported only with a certificate checked in FP64:
 * a Farkas vector, or a dual value of the polish's multipliers above every
 * objective value in the box that the chained velocity rows give (weak
 * duality).  Paths are launched in groups by segment count; each group runs
 * twice: every path first with a small working set, then the few whose
 * working set outgrew it at the full size, continuing from the working set
 * the first launch held (their outputs are rewritten; until then status_out
 * may hold an internal value).  The groups run on `stream` and the device's
 * side streams (see the conventions at the top), ordered after what `stream`
 * holds and before what it gets next.
 *   x0 [N][6], goal [N][3]; opts as for rbp_solve_batch (plain and
 *   store_for_backward are ignored);
 *   P_out [3 points_total]: the control points of every segment (NaN unless
 *   SOLVED); cost_out, status_out, kkt_out [N]; iters_out [N][2] or NULL
 *   (ADMM iterations, polish steps).
 * Errors: RBP_E_INVALID, RBP_E_DEVICE.
 */
int rbp_solve_chains(rbp_chains* chains, const double* x0, const double* goal, const rbp_solve_opts* opts,
                     double* P_out, double* cost_out, int32_t* status_out, double* kkt_out,
                     int32_t* iters_out, hipStream_t stream);

/* Releases a path batch (no-op for NULL). */
void rbp_destroy_chains(rbp_chains* chains);

/* ------------------------------------------------------------------------
 * Cutting graph edges against obstacles (Sec. III-B, Alg. 2, eq. Cut-QP).
 *
 * A pair is an edge, the control points P of its degree-p Bezier curve, and
 * a convex obstacle O (Assumption 1): an axis-aligned box lo <= x <= hi, or a
 * convex polytope {x : A x <= b} of n_c halfspaces.  By the convex-hull
 * property (Property 1) the curve is free of O when conv(P) and O are
 * disjoint.  Each pair runs Alg. 2: (1) a control point inside O -> may
 * collide; (2) every control point strictly beyond the supporting plane of O
 * whose normal points from the point of O nearest the centroid of P to that
 * centroid -> free; (3) otherwise the Cut-QP
 *     min |delta|^2  over convex weights lam and slacks delta,
 *     A P^T lam <= b + delta,
 * free when its optimum |delta*|^2 is positive.  For a box (unit rows) the
 * optimum is the squared distance between conv(P) and the box; for a
 * polytope it is min over conv(P) of |(A x - b)_+|^2.  Step 3 decides
 * free / may collide by the distance between conv(P) and O (GJK: zero
 * exactly when the Cut-QP optimum is zero; below 1e-24 max(1, |P|)^2 counts
 * as zero).  When qp_dist2 is given, a second pass computes the optimum of
 * each undecided polytope pair exactly (Newton steps over the pieces of the
 * objective, each piece minimised by Wolfe's minimum-norm-point method),
 * certified by the Lagrange-dual gap.
 * ------------------------------------------------------------------------ */
#define RBP_CUT_MAX_POLY_ROWS 32   /* halfspaces per polytope obstacle            */
#define RBP_CUT_MAX_POLY_VERTS 64  /* vertices per polytope obstacle              */

typedef struct rbp_cut_desc {
  int32_t n_edges;            /* >= 0                                         */
  int32_t n_obstacles;        /* box obstacles, >= 0                          */
  int32_t degree;             /* 1..RBP_MAX_DEGREE, the same for every edge    */
  int32_t reserved;           /* 0                                            */
  const double* box_lo;       /* device [n_obstacles][3]                      */
  const double* box_hi;       /* device [n_obstacles][3], hi >= lo             */
  /* Polytope obstacles, numbered n_obstacles .. n_obstacles + n_polytopes - 1
   * in the outputs.  Each must be bounded with a non-empty interior (a
   * convex polytope); rbp_build_cut checks this (RBP_E_SHAPE otherwise). */
  int32_t n_polytopes;        /* >= 0                                         */
  int32_t reserved2;          /* 0                                            */
  const int32_t* pob_off;     /* device [n_polytopes+1]: polytope j owns rows
                                 pob_off[j] .. pob_off[j+1]-1, pob_off[0] = 0,
                                 4..RBP_CUT_MAX_POLY_ROWS rows each            */
  const double* pob_A;        /* device [rows][3] outward normals (non-zero)  */
  const double* pob_b;        /* device [rows]: the polytope is A x <= b       */
} rbp_cut_desc;

typedef struct rbp_cut rbp_cut;

/* Upper bound on n_edges * (n_obstacles + n_polytopes) (the undecided-pair
 * list is sized for every pair). */
#define RBP_CUT_MAX_PAIRS (1LL << 28)

/*
 * Keeps the obstacle arrays (device pointers, owned by the caller, which
 * must keep them alive) and allocates the undecided-pair list.  Polytope
 * rows are copied to the host (the call synchronises `stream`) to enumerate
 * each polytope's vertices (intersections of three of its planes that
 * satisfy every row, duplicates merged), which the supporting planes and the
 * distance of step 3 use; the vertex table is uploaded and owned by the
 * object.
 * Errors: RBP_E_INVALID (null pointers, negative counts, reserved fields not
 * 0), RBP_E_SHAPE (degree out of range, more than RBP_CUT_MAX_PAIRS pairs,
 * row counts out of range, a zero or non-finite row, a polytope that is
 * unbounded, empty or flat, or with more than RBP_CUT_MAX_POLY_VERTS
 * vertices), RBP_E_ALLOC, RBP_E_DEVICE.
 */
int rbp_build_cut(const rbp_cut_desc* desc, hipStream_t stream, rbp_cut** out);

/*
 * Classifies every (edge, obstacle) pair; stream-ordered, asynchronous.
 *   P          device [n_edges][degree+1][3] control points (point-major)
 *   code       device [n_obst][n_edges] uint8: 1 free, 0 may collide, with
 *              n_obst = n_obstacles + n_polytopes (boxes first)
 *   step       nullable, same shape: the step of Alg. 2 that decided (1, 2, 3)
 *   qp_dist2   nullable, same shape, double: the Cut-QP optimum |delta*|^2
 *              where step 3 ran, NaN where the heuristic decided
 *   n_collide  device [n_edges] int32: obstacles the edge may collide with
 *              (0 = the edge stays in the cut graph)
 * Codes are obstacle-major: pair (e, o) is at o * n_edges + e.
 * Errors: RBP_E_INVALID (null pointers), RBP_E_DEVICE.
 */
int rbp_cut_run(rbp_cut* cut, const double* P, uint8_t* code, uint8_t* step, double* qp_dist2,
                int32_t* n_collide, hipStream_t stream);

/* Number of pairs the last rbp_cut_run sent to step 3 (synchronises the
 * stream of that run).  Errors: RBP_E_INVALID, RBP_E_DEVICE. */
int rbp_cut_qp_count(rbp_cut* cut, int64_t* n_qp);

/* Frees the list (waits for the last run). */
void rbp_destroy_cut(rbp_cut* cut);

/* ------------------------------------------------------------------------
 * Building the graph (Sec. III-A, Thm. 2) and adjacent hyperplanes
 * (Alg. 2, Sec. III-D).
 *
 * With the reachable-polytope pair (F, G) of Theorem 2 split into the
 * columns acting on the start node (F1) and on the end node (F2), nodes v_i
 * and v_j are joined by the edge i -> j when F1 v_i + F2 v_j <= G (every
 * row); a node is not joined to itself.  Numbering the nodes along a
 * space-filling curve lets the kernel skip whole tiles of far-apart pairs
 * (an exact bound); the result does not depend on the numbering.
 * ------------------------------------------------------------------------ */
#define RBP_GRAPH_MAX_DIM 12
#define RBP_GRAPH_MAX_ROWS 1024
#define RBP_GRAPH_MAX_NODES (1 << 20)

typedef struct rbp_graph_desc {
  int32_t n_nodes;            /* 0..RBP_GRAPH_MAX_NODES                        */
  int32_t dim;                /* node state dimension, 1..RBP_GRAPH_MAX_DIM     */
  int32_t n_rows;             /* rows m of F, 1..RBP_GRAPH_MAX_ROWS             */
  int32_t reserved;           /* 0                                             */
  const double* F1;           /* device [m][dim], kept by pointer              */
  const double* F2;           /* device [m][dim]                               */
  const double* G;            /* device [m]                                    */
} rbp_graph_desc;

typedef struct rbp_graph rbp_graph;

/* Keeps (F1, F2, G) by pointer (the caller keeps them alive) and allocates
 * the per-node workspace (2 n m doubles plus tile bounds).  Errors:
 * RBP_E_INVALID, RBP_E_SHAPE (sizes out of range), RBP_E_ALLOC. */
int rbp_build_graph(const rbp_graph_desc* desc, hipStream_t stream, rbp_graph** out);

/*
 * Adjacency of the nodes V (device [n_nodes][dim]); stream-ordered.
 *   adj     device [n_nodes][ceil(n_nodes / 32)] uint32: bit (j % 32) of word
 *           (j / 32) in row i is the edge i -> j
 *   degree  device [n_nodes] int32: out-degree
 * Errors: RBP_E_INVALID (null pointers), RBP_E_DEVICE.
 */
int rbp_graph_run(rbp_graph* graph, const double* V, uint32_t* adj, int32_t* degree, hipStream_t stream);

void rbp_destroy_graph(rbp_graph* graph);

/*
 * rbp_graph_run without a graph object and without any device allocation,
 * for callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same result as rbp_build_graph +
 * rbp_graph_run + rbp_destroy_graph on `desc`, bit for bit.
 *   desc     host pointer; F1, F2, G device pointers as in rbp_graph_desc,
 *            read during the call only
 *   V, adj, degree   as in rbp_graph_run (caller-owned device buffers)
 * Workspace: a fixed device array of RBP_GRAPH_NOALLOC_DOUBLES doubles
 * (8 MiB) per GPU, held by the library until the process ends; a call needs
 * 2 n m + 2 ceil(n / 64) m of them (n nodes, m rows; 5,000 nodes with 64 rows
 * need 650,112).  Every call on one GPU uses that GPU's array, so calls that
 * overlap on one GPU (different streams, or host threads) race: order them
 * on one stream.  Nothing in the workspace must start at zero (each call
 * overwrites what it reads).  The first call on a device looks up the
 * array's address (hipGetSymbolAddress) and caches it.
 * Errors: RBP_E_INVALID (null pointers, reserved != 0), RBP_E_SHAPE (sizes
 * out of the ranges of rbp_build_graph), RBP_E_SCRATCH (the workspace is
 * too small for n and m; checked before any device call), RBP_E_DEVICE.
 */
#define RBP_GRAPH_NOALLOC_DOUBLES (1 << 20)
int rbp_graph_run_noalloc(const rbp_graph_desc* desc, const double* V, uint32_t* adj, int32_t* degree,
                          hipStream_t stream);

/*
 * adjacentHyperplane for n nodes X (device [n][3]) against axis-aligned
 * boxes (device [n_obstacles][3] each): the nearest box (Euclidean distance,
 * lowest index on ties; -1 when there is none), the closest point on it,
 * and the plane through that point with unit normal toward the node:
 *   box_index [n] int32, point [n][3], plane [n][4] = (n_x, n_y, n_z, l):
 *   the box lies in n.y <= l and the node in n.x > l (n = 0, l = 0 for a
 *   node inside a box).  Stream-ordered.  Errors: RBP_E_INVALID, RBP_E_DEVICE.
 */
int rbp_adjacent_hyperplanes(int32_t n_nodes, const double* X, int32_t n_obstacles, const double* box_lo,
                             const double* box_hi, int32_t* box_index, double* point, double* plane,
                             hipStream_t stream);

/*
 * Batched MPC refinement (eq. MPC, Sec. III-D).  Each instance refines a
 * path over a horizon of N steps of length dt for the double integrator in
 * R^3 (state x = (position p, velocity v), input u = acceleration, exact
 * zero-order-hold discretisation x_{k+1} = A x_k + B u_k):
 *
 *   minimise   sum_{k=1}^{N-1} (x_k - r_k)' Q (x_k - r_k)
 *            + sum_{k=0}^{N-1} u_k' R u_k + w |p_{k+1} - p_k|^2
 *   subject to x_0 = x0,  x_N = r_N,  dynamics,
 *              F1 x_k + F2 x_{k+1} <= G          (reachable rows, Thm. 2)
 *              n_k . P_j >= l_k,  j = 0..3        (keep-out plane of step k)
 *
 * where P_j are the control points of the cubic Bezier curve on [0, dt]
 * joining the two states (Lemma 1): p_k, p_k + dt/3 v_k, p_{k+1} - dt/3
 * v_{k+1}, p_{k+1}; by the convex-hull property the whole step stays on the
 * free side of the plane.  The planes (one per step) come from the adjacent
 * hyperplanes of the reference nodes (rbp_adjacent_hyperplanes): one SQP
 * iteration, as in Sec. IV.
 *
 * Solver: one wavefront per instance, primal-dual interior point in FP64
 * with Riccati-structured Newton systems.  Instances are independent.
 */
#define RBP_MPC_MAX_HORIZON 64
#define RBP_MPC_MAX_REACH 32

typedef struct rbp_mpc_desc {
  int32_t n_instances;        /* >= 0                                            */
  int32_t horizon;            /* N, 2..RBP_MPC_MAX_HORIZON                       */
  int32_t n_reach;            /* m reachable rows per step, 0..RBP_MPC_MAX_REACH  */
  int32_t reserved;           /* must be 0                                       */
  double dt;                  /* step, > 0                                       */
  double Q[36];               /* tracking weight (6 x 6, row-major, symmetric
                                 positive semidefinite; host values)             */
  double R[9];                /* input weight (3 x 3, symmetric positive
                                 definite; host values)                          */
  double w_length;            /* weight of |p_{k+1} - p_k|^2, >= 0                */
  const double* F1;           /* [m][6] device: rows on x_k                      */
  const double* F2;           /* [m][6] device: rows on x_{k+1}                  */
  const double* G;            /* [m] device                                      */
} rbp_mpc_desc;

typedef struct rbp_mpc rbp_mpc;

/* Validates the description, copies F1, F2, G to the host (the call
 * synchronises `stream`), prepares the per-step constants and uploads them.
 * Errors: RBP_E_INVALID (null pointers with m > 0, reserved != 0, dt <= 0,
 * w < 0, Q not symmetric or with a negative diagonal, R not symmetric
 * positive definite), RBP_E_SHAPE (horizon or m out of range, a reachable row
 * that vanishes once x_{k+1} is written through the dynamics), RBP_E_ALLOC,
 * RBP_E_DEVICE. */
int rbp_build_mpc(const rbp_mpc_desc* desc, hipStream_t stream, rbp_mpc** out);

/*
 * Solves every instance.
 *   x0      [n][6]        start states
 *   ref     [n][N+1][6]   reference states r_0..r_N (r_N is the terminal state)
 *   planes  [n][N][4]     (n_k, l_k) per step; n_k need not be unit length
 *   max_iters             interior-point iteration cap (> 0; 40 is ample)
 *   tol                   target of the average complementarity (> 0;
 *                         1e-15 is the default of the Python binding); the
 *                         primal residual of the unit rows must also reach
 *                         1e-10 and the dual residual 1e-8 (1 + gradient
 *                         scale)
 *   X       [n][N+1][6]   states (X_N from the dynamics of the last step)
 *   U       [n][N][3]     inputs
 *   cost    [n]           objective value
 *   status  [n]           RBP_SOLVED (scaled KKT residual of the returned
 *                         point <= 1e-6), RBP_INFEASIBLE (a certificate
 *                         checked in FP64: with the last multipliers w >= 0
 *                         and a least-squares terminal costate, the affine
 *                         function sum w_i (row_i - bound_i) + pi'(x_N - r_N)
 *                         of the inputs is positive over the whole input box
 *                         that the rows acting on u alone allow; X, U NaN,
 *                         cost +inf), RBP_MAXITER (stopped before a KKT
 *                         residual <= 1e-6 without such a certificate:
 *                         iteration cap or a Newton system that broke down;
 *                         also every infeasible instance when no row bounds
 *                         the inputs alone), RBP_NUMERICAL (converged by the
 *                         tolerances above, residual still above 1e-6),
 *                         RBP_INVALID_INPUT (non-finite input or a zero
 *                         plane normal; X, U, cost are NaN).  Otherwise X,
 *                         U, cost hold the last iterate.
 *   kkt     [n]           max of the scaled primal, dual (least-squares
 *                         costates) and complementarity residuals
 *   iters   [n] or NULL   interior-point iterations
 * Errors: RBP_E_INVALID (null pointer, max_iters <= 0, tol <= 0),
 * RBP_E_DEVICE.
 */
int rbp_mpc_solve(rbp_mpc* mpc, const double* x0, const double* ref, const double* planes, int32_t max_iters,
                  double tol, double* X, double* U, double* cost, int32_t* status, double* kkt, int32_t* iters,
                  hipStream_t stream);

/* Releases the solver (no-op for NULL); synchronises its last stream first. */
void rbp_destroy_mpc(rbp_mpc* mpc);

/* Static string for a call result or per-instance status code. */
const char* rbp_status_string(int code);

#ifdef __cplusplus
}
#endif
#endif /* RBP_H_ */
