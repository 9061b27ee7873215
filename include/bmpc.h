/*
 * bmpc.h -- C ABI of the MI355X branch-MPC hot path (libbmpc.so).
 *
 * The library solves branch model predictive control (BMPC) problems on a
 * trajectory tree with an augmented-Lagrangian multiple-shooting iLQR whose
 * inner step is a tree LQR (Riccati recursion with an exact merge of the
 * children's value functions at every branching node).
 *
 * General conventions
 *  - Every call returns a bmpc_status.  BMPC_OK = 0.  On failure,
 *    bmpc_last_error() returns a thread-local message (with the node id for
 *    BMPC_ERR_NOT_PD).
 *  - Opaque handles (bmpc_tree, bmpc_lqr_plan, bmpc_problem, bmpc_batch,
 *    bmpc_mlp) are owned by the library: every *_create has a *_destroy.
 *  - Arrays passed to the library are owned by the caller.  Each argument
 *    states whether it is a host pointer or a device pointer (device = HBM
 *    memory of the current HIP device, e.g. torch.Tensor.data_ptr()).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *    that take a stream are asynchronous on it unless stated otherwise.
 *  - Handles are not thread-safe; separate handles are independent.
 *  - All floating point is FP64 except the warm-starter network (BF16
 *    weights and activations, FP32 accumulation and master weights).
 *
 * Trees
 *  parent[0] = -1, 0 <= parent[i] < i, and parent[] non-decreasing for i >= 1.
 *  This is the stage-major breadth-first order: the nodes of one stage are
 *  contiguous and the children of one node are contiguous.  Other orders are
 *  rejected with BMPC_ERR_TOPOLOGY (a tree in another order goes through
 *  bmpc_tree_create_any and bmpc_tree_permute).  The stage of a node is its depth; a
 *  leaf is a node with no children; "control nodes" are all other nodes.
 *  Dynamics are stored on the edge, i.e. at the child: (A_j, B_j, c_j) at
 *  node j describe x_j = A_j x_{p(j)} + B_j u_{p(j)} + c_j.  Entries of the
 *  root (j = 0) are ignored.
 *
 * Matrix layouts (per plan; see bmpc_lqr_plan_create)
 *  BMPC_LAYOUT_NODE_MAJOR: entry (r, c) of the matrix of node i at
 *      X[(i * rows + r) * cols + c]   (each node's matrix contiguous, row-major)
 *  BMPC_LAYOUT_ELEM_MAJOR: entry (r, c) of the matrix of node i at
 *      X[(r * cols + c) * N + i]      (structure of arrays: one array per entry)
 *  Vectors follow the same rule with cols = 1.
 */
#ifndef BMPC_H
#define BMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BMPC_API __attribute__((visibility("default")))

typedef int32_t bmpc_status;
enum {
    BMPC_OK = 0,
    BMPC_ERR_INVALID_ARG = 1,
    BMPC_ERR_TOPOLOGY = 2,
    BMPC_ERR_NOT_PD = 3,     /* a Riccati Hessian H_n was not positive definite */
    BMPC_ERR_NONFINITE = 4,  /* NaN/Inf met in the iteration */
    BMPC_ERR_MAXITER = 5,    /* iteration cap reached; outputs hold the last iterate */
    BMPC_ERR_LINESEARCH = 6, /* no step size accepted several times in a row */
    BMPC_ERR_HIP = 7,        /* a HIP runtime call failed */
    BMPC_ERR_OOM = 8,        /* device or host allocation failed */
    BMPC_ERR_UNSUPPORTED = 9 /* dimension or variant not built into this library */
};

enum { BMPC_LAYOUT_NODE_MAJOR = 0, BMPC_LAYOUT_ELEM_MAJOR = 1 };

/* bmpc_settings.block_size value: one problem solved by the whole grid. */
enum { BMPC_BLOCK_GRID = -1 };

/* Backward-pass variants of the tree LQR. */
enum {
    BMPC_RICCATI_AUTO = 0,
    /* level-parallel: every node of one depth is processed at the same time;
       branch nodes are merged by the last child to finish (no grid barrier) */
    BMPC_RICCATI_LEVEL = 1,
    /* log-depth: associative scan of conditional value functions along each
       unbranched segment, exact merges at branching nodes */
    BMPC_RICCATI_SEGSCAN = 2
};

/* Message of the last failed call on this thread ("" if none). */
BMPC_API const char* bmpc_last_error(void);
/* Library version: major*10000 + minor*100 + patch. */
BMPC_API int32_t bmpc_version(void);
/* Number of HIP devices visible to the library (0 if none).  Host only; it
   touches the HIP runtime. */
BMPC_API int32_t bmpc_device_count(void);

/* ------------------------------------------------------------------------
 * Topology: tree index sets of the problem statement (Sec. II-B): parent
 * p(i), children ch(i), stage sets N_k, leaves L.
 * ---------------------------------------------------------------------- */
typedef struct bmpc_tree bmpc_tree;

/* parent: host pointer, num_nodes entries, order rules above.  The tree is
   analysed on the host (stages, children, maximal unbranched segments,
   root-to-leaf paths) and uploaded to the current device. */
BMPC_API bmpc_status bmpc_tree_create(const int32_t* parent, int32_t num_nodes, bmpc_tree** out);
BMPC_API void bmpc_tree_destroy(bmpc_tree* tree);
/* Host outputs; any pointer may be NULL.  depth = largest stage;
   num_segments = number of maximal unbranched segments (a segment starts at
   the root or at a child of a node with >= 2 children and ends at a leaf or
   at a node with >= 2 children). */
BMPC_API bmpc_status bmpc_tree_info(const bmpc_tree* tree, int32_t* num_nodes, int32_t* num_leaves,
                                    int32_t* depth, int32_t* num_segments);
/* Segment id of every node (host output, num_nodes entries); segments are
   numbered by increasing start node. */
BMPC_API bmpc_status bmpc_tree_segments(const bmpc_tree* tree, int32_t* seg_of_node);
/* Node probability weights: pi_n = total probability of the leaves below n.
   leaf_prob: host, one entry per leaf in increasing node order.
   node_weight: host output, num_nodes entries. */
BMPC_API bmpc_status bmpc_weights_from_probs(const bmpc_tree* tree, const double* leaf_prob,
                                             double* node_weight);

/* Trees in the caller's own node order (the index sets of Sec. II-B fix
   none).  parent: host, num_nodes entries; exactly one node has parent -1
   (the root), every other node's parent is another node's index, and every
   node descends from the root (else BMPC_ERR_TOPOLOGY, e.g. for a parent
   cycle).  The library's order is the breadth-first order from the root
   with each node's children in increasing caller index.
   bmpc_tree_order writes order[k] = caller index of library node k (host
   output, num_nodes entries) and, if lib_parent is not NULL, the parent
   array in the library's order (host output, num_nodes entries; it
   satisfies the rules above and can be given to bmpc_tree_create).  On
   error the outputs are unspecified.  Host only. */
BMPC_API bmpc_status bmpc_tree_order(const int32_t* parent, int32_t num_nodes, int32_t* order,
                                     int32_t* lib_parent);
/* bmpc_tree_create for a parent array in any order (rules of
   bmpc_tree_order).  The tree keeps the permutation for bmpc_tree_permute;
   order (host output, nullable) receives it as in bmpc_tree_order.  Node k
   of every other call on this tree is library node k. */
BMPC_API bmpc_status bmpc_tree_create_any(const int32_t* parent, int32_t num_nodes, int32_t* order,
                                          bmpc_tree** out);
enum { BMPC_TO_LIBRARY_ORDER = 0, BMPC_TO_CALLER_ORDER = 1 };
/* Moves per-node data between the caller's node order and the library's:
   BMPC_TO_LIBRARY_ORDER gathers dst[library node k] = src[caller node
   order[k]], BMPC_TO_CALLER_ORDER scatters the other way.  src, dst: device,
   num_nodes x width doubles each in the given layout (BMPC_LAYOUT_*; width =
   rows * cols of one node's entry), caller-owned, distinct and not
   overlapping.  For a tree from bmpc_tree_create the orders agree and the
   call is a device copy.  The first call on a reordered tree allocates
   num_nodes int32 on the current device for the permutation (owned by the
   tree); later calls allocate nothing.  Asynchronous on stream.
   BMPC_ERR_INVALID_ARG for NULL pointers, src == dst, width <= 0 or an
   unknown direction or layout. */
BMPC_API bmpc_status bmpc_tree_permute(bmpc_tree* tree, int32_t direction, int32_t layout,
                                       int32_t width, const double* src, double* dst, void* stream);

/* ------------------------------------------------------------------------
 * Tree LQR (Sec. III, eq. lqr_tree_approx; recursion of eq. tree_Riccati with
 * the gains of eq. tree_feedback_laws; forward rollout of eq.
 * forward_comb_rule along every root-to-leaf path).
 *
 *   min  sum_{n control} 1/2 [x;u]^T [[Q_n, M_n^T],[M_n, R_n]] [x;u] + q_n^T x + r_n^T u
 *      + sum_{l leaf} 1/2 x^T Q_l x + q_l^T x
 *   s.t. x_0 = x0,  x_j = A_j x_{p(j)} + B_j u_{p(j)} + c_j.
 *
 * Outputs: the minimiser (x, u), the costates lam_j = P_j x_j + p_j (the
 * multipliers of the dynamics in the convention L = cost + lam^T (f - x)),
 * and optionally the gains K, k and value functions P, p.
 * ---------------------------------------------------------------------- */
typedef struct bmpc_lqr_plan bmpc_lqr_plan;

/* Allocates device workspace for a tree and dimensions (nx, nu).
   layout: BMPC_LAYOUT_*.  Returns BMPC_ERR_UNSUPPORTED if (nx, nu) has no
   compiled kernel (see bmpc_lqr_supported). */
BMPC_API bmpc_status bmpc_lqr_plan_create(const bmpc_tree* tree, int32_t nx, int32_t nu,
                                          int32_t layout, bmpc_lqr_plan** out);
BMPC_API void bmpc_lqr_plan_destroy(bmpc_lqr_plan* plan);
/* 1 if kernels for (nx, nu, variant) are compiled in, else 0. */
BMPC_API int32_t bmpc_lqr_supported(int32_t nx, int32_t nu, int32_t variant);

/* All array arguments are DEVICE pointers in the plan's layout, N = number of
   nodes.  Sizes: A N*nx*nx, B N*nx*nu, c N*nx (edge data, root ignored);
   Q N*nx*nx, q N*nx (terminal cost at leaves); R N*nu*nu, M N*nu*nx, r N*nu
   (control nodes; leaf entries ignored); x0 nx.  Outputs x N*nx, u N*nu
   (leaf entries set to 0), lam N*nx; K N*nu*nx, k N*nu, P N*nx*nx, p N*nx
   may be NULL (then plan workspace is used).  Inputs and outputs must not
   overlap.  Asynchronous on `stream`.  A non-positive-definite H_n is
   reported by bmpc_lqr_check (the affected outputs are then undefined). */
BMPC_API bmpc_status bmpc_lqr_solve(bmpc_lqr_plan* plan, const double* A, const double* B,
                                    const double* c, const double* Q, const double* R,
                                    const double* M, const double* q, const double* r,
                                    const double* x0, double* x, double* u, double* lam,
                                    double* K, double* k, double* P, double* p, int32_t variant,
                                    void* stream);
/* bmpc_lqr_solve for HOST arrays (Sec. III, eq. lqr_tree_approx): A ... r,
   x0 inputs and x, u, lam outputs are caller-owned host pointers with the
   sizes and the plan's layout of bmpc_lqr_solve; no gains or value
   functions are returned.  The call packs the inputs into a pinned host
   block, copies it to the device in one transfer, runs the same kernels on
   `stream`, copies x, u, lam back in one transfer and synchronises the
   stream before it returns (blocking).  The first call on a plan allocates
   the pinned and device staging blocks (N (2 nx^2 + 2 nx nu + nu^2 + 4 nx +
   2 nu) + nx doubles each, owned by the plan); later calls allocate
   nothing.  Errors as bmpc_lqr_solve, BMPC_ERR_OOM if a staging block
   cannot be allocated; positive definiteness is reported by
   bmpc_lqr_check. */
BMPC_API bmpc_status bmpc_lqr_solve_host(bmpc_lqr_plan* plan, const double* A, const double* B,
                                         const double* c, const double* Q, const double* R,
                                         const double* M, const double* q, const double* r,
                                         const double* x0, double* x, double* u, double* lam,
                                         int32_t variant, void* stream);
/* The same solve in FP32 (the single-precision variant of the recursion,
   Sec. V-A): float arrays of the sizes and layout above.  Compiled for the
   dimensions whose FP64 solve uses one lane per node (nx <= 6); others
   return BMPC_ERR_UNSUPPORTED.  The first FP32 or mixed-precision call on a
   plan allocates the plan's FP32 workspace (so it cannot be captured in a
   graph); later calls allocate nothing.  Positive definiteness is reported
   by bmpc_lqr_check as for the FP64 solve. */
BMPC_API bmpc_status bmpc_lqr_solve_f32(bmpc_lqr_plan* plan, const float* A, const float* B, const float* c,
                                        const float* Q, const float* R, const float* M, const float* q,
                                        const float* r, const float* x0, float* x, float* u, float* lam, float* K,
                                        float* k, float* P, float* p, void* stream);

#define BMPC_LQR_REFINE_MAX 64
/* Mixed precision: the FP64 problem of bmpc_lqr_solve (same arrays, sizes
   and layout) solved by FP32 Riccati sweeps with FP64 iterative refinement.
   The matrices are rounded to FP32 once; then 1 + refine_steps FP32 solves
   each take as linear terms the FP64 KKT residual of the current FP64
   iterate (x, u, lam) -- stationarity in u and x and the dynamics defects,
   with the convention of the costates above -- and add their solution to
   it.  Each step shrinks the error by about cond * 2^-24, so a few steps
   reach FP64 accuracy on well-conditioned trees; ill-conditioned ones
   converge slowly or not at all, which res_norms shows.
   refine_steps: 0 .. BMPC_LQR_REFINE_MAX.
   res_norms: DEVICE array of refine_steps + 2 doubles, or NULL; entry i is
   the largest |KKT residual row| after i FP32 solves (entry 0: of the data,
   i.e. at x = u = lam = 0).  Asynchronous on `stream`; bmpc_lqr_check
   reports the positive-definiteness status of the last FP32 solve.
   Returns BMPC_ERR_UNSUPPORTED where bmpc_lqr_solve_f32 does. */
BMPC_API bmpc_status bmpc_lqr_solve_mixed(bmpc_lqr_plan* plan, const double* A, const double* B, const double* c,
                                          const double* Q, const double* R, const double* M, const double* q,
                                          const double* r, const double* x0, double* x, double* u, double* lam,
                                          int32_t refine_steps, double* res_norms, void* stream);

/* Synchronises `stream` and reports the numerical status of the last solve
   on this plan: BMPC_OK, or BMPC_ERR_NOT_PD with *bad_node set (smallest
   failing node id).  bad_node may be NULL. */
BMPC_API bmpc_status bmpc_lqr_check(bmpc_lqr_plan* plan, int32_t* bad_node, void* stream);

/* ------------------------------------------------------------------------
 * Branch-MPC problem (Sec. II-B, eq. bmpc) for a kinematic bicycle.
 *
 * State x = [px, py, psi, v], input u = [a, delta].  Dynamics: one RK4 step
 * of  d/dt x = [v cos psi, v sin psi, v tan(delta)/L, a]  over dt with the
 * input held.  Node cost: w_n * (1/2 (x - ref_n)^T diag(Qd) (x - ref_n)
 * + 1/2 u^T diag(Rd) u) at control nodes, w_n * 1/2 (x - ref_n)^T diag(Qd)
 * (x - ref_n) at leaves.  Constraints g <= 0 in five slots per node:
 * a - a_max, -a - a_max, delta - steer_max, -delta - steer_max (control
 * nodes), and obs_radius - |(px, py) - o_n| at nodes with an obstacle.
 * ---------------------------------------------------------------------- */
typedef struct {
    double wheelbase, dt;
    double Qd[4], Rd[2];
    double a_max, steer_max, obs_radius;
} bmpc_bicycle_params;

/* Parameters of the AL outer loop and iLQR inner loop (Alg. 1).  Defaults
   from bmpc_settings_default: eps_tol 1e-6, tau 100, omega0 1, eta0 0.1,
   a_omega = b_omega = 1, a_eta 0.1, b_eta 0.9, rho0 100, mu0 100, Armijo
   constant 1e-4, n_alpha 10 step sizes 2^0 .. 2^-9 per backtracking round,
   ls_rounds 3, max_outer 50, max_inner 100 (per outer iteration),
   max_ls_fail 3 consecutive line-search failures, Gauss-Newton Hessian
   (eig_floor 1e-9 for the exact one).  The merit of a trial
   point whose steering angle leaves (-pi/2, pi/2), where the bicycle model is
   undefined, is +inf.  Tolerances omega and eta are floored at eps_tol. */
typedef struct {
    double eps_tol, tau, omega0, eta0, a_omega, b_omega, a_eta, b_eta;
    double rho0, mu0, armijo_beta;
    int32_t n_alpha, max_outer, max_inner, max_ls_fail, riccati_variant;
    /* threads per problem in batched solves: 64, 128 or 256; 0 = the value
       chosen by bmpc_batch_tune for the batch, else 256, except that a batch
       of one problem of at least 16,384 nodes is solved by the whole grid;
       BMPC_BLOCK_GRID = the whole grid (cooperative launch, level-parallel
       backward pass; batches of one problem only) */
    int32_t block_size;
    /* cap on inner iterations summed over all outer iterations (0 = none);
       reaching it ends the solve with BMPC_ERR_MAXITER */
    int32_t max_iter_total;
    /* backtracking rounds of the line search (Sec. IV-A), 1 .. 8: round k
       tries the n_alpha step sizes 2^-(k n_alpha) .. 2^-(k n_alpha + n_alpha
       - 1) and runs only when round k - 1 accepted none; if no round accepts
       a step, the step 2^-(ls_rounds n_alpha - 1) is taken and counted as a
       line-search failure */
    int32_t ls_rounds;
    /* Hessian of the quadratic model (Sec. IV-A): BMPC_HESSIAN_GAUSS_NEWTON
       (dynamics and constraint curvature dropped), or BMPC_HESSIAN_EXACT:
       the Hessian of the Lagrangian per node -- with the curvature of the
       active obstacle penalty and the dynamics curvature contracted with the
       children's multipliers, which gives a cross block M -- whose
       eigenvalues are raised to at least eig_floor (> 0) times
       max(1, the block's largest |eigenvalue|). */
    int32_t hessian;
    double eig_floor;
} bmpc_settings;
enum { BMPC_HESSIAN_GAUSS_NEWTON = 0, BMPC_HESSIAN_EXACT = 1 };

/* Result of one solve.  r_kkt: last KKT residual of the relaxed problem
   (infinity norm of the Lagrangian gradient and of the defects); viol:
   constraint violation max |max(g, -y/rho)|; start: 1 if the solve began
   from the caller's start point, 0 if from the cold start.  time_ms: device
   time of the solve's phases, summed over its inner iterations, read from
   the constant-rate device clock by the solving team's first thread:
   [BMPC_PHASE_LINEARISE] linearisation, quadratisation and KKT residual,
   [BMPC_PHASE_BACKWARD] backward Riccati, [BMPC_PHASE_FORWARD] forward
   rollout, [BMPC_PHASE_LINESEARCH] merit slope and line search,
   [BMPC_PHASE_UPDATE] step update and the outer (BCL) update.  The start
   point (rollout, adjoint sweep) is not included. */
enum {
    BMPC_PHASE_LINEARISE = 0,
    BMPC_PHASE_BACKWARD = 1,
    BMPC_PHASE_FORWARD = 2,
    BMPC_PHASE_LINESEARCH = 3,
    BMPC_PHASE_UPDATE = 4,
    BMPC_NUM_PHASES = 5
};
typedef struct {
    int32_t status, outer_it, inner_it, ls_failures, bad_node, start;
    double r_kkt, viol, rho, mu, merit;
    double time_ms[BMPC_NUM_PHASES];
} bmpc_stats;

typedef struct bmpc_problem bmpc_problem;
typedef struct bmpc_batch bmpc_batch;

BMPC_API void bmpc_settings_default(bmpc_settings* s);
BMPC_API void bmpc_bicycle_default(bmpc_bicycle_params* p);

/* Node references for lane following: ref_n = [speed*dt*stage, ybar_n, 0,
   speed] with ybar_n the leaf_prob-weighted mean of leaf_offset over the
   leaves below n.  leaf_prob, leaf_offset: host, one entry per leaf in node
   order; node_ref: host output, N x 4. */
BMPC_API bmpc_status bmpc_node_refs(const bmpc_tree* tree, const double* leaf_prob, const double* leaf_offset,
                                    double dt, double speed, double* node_ref);

/* All arrays HOST pointers, node-major: node_weight N, node_ref N x 4,
   node_obs N x 2 (obstacle centre used by the node), has_obs N (0/1), x0 4.
   Copied to the current device.  Non-finite data -> BMPC_ERR_NONFINITE. */
BMPC_API bmpc_status bmpc_problem_create(bmpc_tree* tree, const bmpc_bicycle_params* prm,
                                         const double* node_weight, const double* node_ref,
                                         const double* node_obs, const int32_t* has_obs, const double* x0,
                                         bmpc_problem** out);
BMPC_API void bmpc_problem_destroy(bmpc_problem* problem);
/* New measured state (host pointer, 4 entries). */
BMPC_API bmpc_status bmpc_problem_set_x0(bmpc_problem* problem, const double* x0);
/* Replace all data of a problem on the same tree (host arrays as in
   bmpc_problem_create; synchronous).  Batches holding the problem see the
   new data at their next launch. */
BMPC_API bmpc_status bmpc_problem_update(bmpc_problem* problem, const double* node_weight,
                                         const double* node_ref, const double* node_obs,
                                         const int32_t* has_obs, const double* x0);
/* Current measured state (host output, 4 entries; synchronous).  Reflects
   bmpc_batch_shift, which advances it on the device. */
BMPC_API bmpc_status bmpc_problem_get_x0(const bmpc_problem* problem, double* x0);
/* Number of warm-start network outputs the problem takes (see
   bmpc_batch_start_from_network): 6 per control node + 1 per node with an
   obstacle. */
BMPC_API bmpc_status bmpc_problem_output_width(const bmpc_problem* problem, int32_t* width);

/* Solve one problem (Alg. 1).  x (N x 4), u (N x 2), lam (N x 4, multipliers
   of the dynamics, convention L = L_a + lam^T (f - x)), ye (N x 5, PHR
   multiplier estimates): DEVICE pointers, node-major, written on return.
   warm bits: 1 = start from the given x, u; 8 = start from the given u with
   x from the exact rollout from x0 (wins over 1); 2 = given lam; 4 = given
   ye (clamped at zero); 16 = guarded: also form the cold start and keep it
   instead if its max(KKT residual, violation) at rho0 is smaller than the
   given start's (stats->start tells which was used).  Without bits 1 and 8
   the start is u = 0 with the exact rollout from x0; without bit 2 lam comes
   from the adjoint sweep at the start point.  Synchronous:
   returns after the solve with *stats (host) filled.  Returns the solver
   status (BMPC_ERR_MAXITER / _LINESEARCH / _NONFINITE / _NOT_PD with the
   last iterate in the outputs). */
BMPC_API bmpc_status bmpc_solve(bmpc_problem* problem, const bmpc_settings* s, int32_t warm, double* x,
                                double* u, double* lam, double* ye, bmpc_stats* stats, void* stream);

/* Linearisation and Gauss-Newton quadratisation at a given point (Sec.
   IV-A): per node n, A (N x 16) and B (N x 8) = Jacobians of the RK4 step at
   (x_n, u_n) (rows of leaves are zero), c (N x 4) = defect of the edge into
   n, f(x_p, u_p) - x_n (zero at the root), Q (N x 16), R (N x 4), q (N x 4),
   r (N x 2) = Gauss-Newton Hessian blocks and gradient of the augmented
   objective.  Inputs and outputs DEVICE pointers, node-major.  kkt_viol
   (host, 2 entries, nullable) receives the KKT residual and the constraint
   violation.  Synchronous if kkt_viol is given, otherwise asynchronous. */
BMPC_API bmpc_status bmpc_linearize(bmpc_problem* problem, const double* x, const double* u,
                                    const double* lam, const double* ye, double rho, double* A, double* B,
                                    double* c, double* Q, double* R, double* q, double* r, double* kkt_viol,
                                    void* stream);

/* The same with the exact Hessian with eigenvalue modification
   (BMPC_HESSIAN_EXACT, relative floor eig_floor > 0): additionally M (N*2*4, the
   cross block d2/du dx per node, zero at leaves); Q and R are the modified
   blocks. */
BMPC_API bmpc_status bmpc_linearize_exact(bmpc_problem* problem, double eig_floor, const double* x,
                                          const double* u, const double* lam, const double* ye, double rho,
                                          double* A, double* B, double* c, double* Q, double* R, double* M,
                                          double* q, double* r, double* kkt_viol, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   linearisation as bmpc_linearize, with its workspace rows in a fixed
   library-owned array of BMPC_NOALLOC_MAX_NODES rows per GPU (3.6 MB, held
   until the process ends) instead of memory allocated for the problem.
   The call allocates nothing.  Arguments as in bmpc_linearize, except
   kkt_viol: a DEVICE pointer (2 doubles, nullable) written by the kernel,
   so the call is always asynchronous on `stream`.  A problem of more than
   BMPC_NOALLOC_MAX_NODES nodes -> BMPC_ERR_INVALID_ARG.  Every call on one
   GPU uses that GPU's one array: calls that overlap on a GPU (different
   streams, or different host threads) race, and the array keeps the last
   call's contents. */
#define BMPC_NOALLOC_MAX_NODES 2048
BMPC_API bmpc_status bmpc_linearize_noalloc(const bmpc_problem* problem, const double* x, const double* u,
                                            const double* lam, const double* ye, double rho, double* A,
                                            double* B, double* c, double* Q, double* R, double* q, double* r,
                                            double* kkt_viol, void* stream);

/* ------------------------------------------------------------------------
 * Batched solve: many independent problems (own trees, own sizes) in one
 * launch.  A persistent kernel: each resident workgroup takes the next
 * problem from a queue (largest first) and solves it start to end, so
 * results do not depend on the schedule; every problem stops on its own
 * convergence.  A batch of one large problem is solved by the whole grid
 * instead (see bmpc_settings.block_size).  The batch owns the state of
 * every problem.
 * ---------------------------------------------------------------------- */
/* problems: host array of `count` handles (they must outlive the batch).
   hist_cap > 0 records per inner iteration [outer, r_kkt, alpha, mu, rho,
   merit] for up to hist_cap iterations per problem. */
BMPC_API bmpc_status bmpc_batch_create(bmpc_problem* const* problems, int32_t count, int32_t hist_cap,
                                       bmpc_batch** out);
BMPC_API void bmpc_batch_destroy(bmpc_batch* batch);
/* Start the solve of every problem (asynchronous on `stream`); warm as in
   bmpc_solve, applied to the state held by the batch. */
BMPC_API bmpc_status bmpc_batch_launch(bmpc_batch* batch, const bmpc_settings* s, int32_t warm, void* stream);
/* Synchronise and copy the `count` results to `stats` (host). */
BMPC_API bmpc_status bmpc_batch_stats(bmpc_batch* batch, bmpc_stats* stats, void* stream);
/* Copy the state of problem i between the batch and DEVICE arrays (node-major
   as in bmpc_solve; NULL parts are skipped): into_batch = 1 writes the batch
   (warm start), 0 reads it.  Asynchronous. */
BMPC_API bmpc_status bmpc_batch_state(bmpc_batch* batch, int32_t i, double* x, double* u, double* lam,
                                      double* ye, int32_t into_batch, void* stream);
/* The same for all problems at once: x (T x 4), u (T x 2), lam (T x 4),
   ye (T x 5) DEVICE arrays, T = bmpc_batch_total_nodes, problems
   concatenated in batch order (problem i starts at row sum_{k<i} N_k).
   NULL parts are skipped.  Asynchronous. */
BMPC_API bmpc_status bmpc_batch_state_all(bmpc_batch* batch, double* x, double* u, double* lam, double* ye,
                                          int32_t into_batch, void* stream);
/* Total number of nodes over all problems of the batch (0 for NULL). */
BMPC_API int64_t bmpc_batch_total_nodes(const bmpc_batch* batch);
/* Receding-horizon step for every problem of the batch, in place: the
   measured state becomes x0' = F(x0, u_0); node n of the next problem stands
   for the old nodes one stage later on the same scenarios (its children), so
   its state, input, costate, PHR multipliers and reference become the
   weight-averaged values of its children; a node whose children are leaves
   repeats its own input; leaves keep costate and multipliers, extrapolate
   the reference from the parent and are rolled out from the new parent.
   The result is the shifted warm start for bmpc_batch_launch(warm = 7).
   The problems' x0 and references are updated.  Asynchronous. */
BMPC_API bmpc_status bmpc_batch_shift(bmpc_batch* batch, void* stream);
/* Shifted warm start of one problem (receding horizon, as bmpc_batch_shift)
   from its previous solution: x (N x 4), u (N x 2), lam (N x 4), ye (N x 5)
   DEVICE arrays, node-major, hold the previous solution on entry and the
   shifted start point on return, for bmpc_solve(warm = 7).  x0_new (host,
   4 entries, nullable): the newly measured state, which becomes the root
   state and the problem's x0; NULL = the predicted F(x0, u_0).  The
   problem's references are shifted with the tree.  Asynchronous.
   Non-finite x0_new -> BMPC_ERR_NONFINITE. */
BMPC_API bmpc_status bmpc_warm_shift(bmpc_problem* problem, double* x, double* u, double* lam, double* ye,
                                     const double* x0_new, void* stream);
/* Start points of problems 0 .. rows-1 from warm-start network outputs.
   Y: DEVICE, rows x width FP32, row-major; row i belongs to problem i:
   first u of every control node in node order (2 each), then the PHR
   multiplier estimate of every active constraint slot in (node, slot)
   order: slots 0-3 (input bounds) of control nodes, slot 4 (obstacle) of
   nodes that carry one.  Writes u and ye of the batch state (leaf inputs
   and inactive slots zero); follow with bmpc_batch_launch(warm = 8 | 4,
   plus 16 to guard against a poor prediction), which rolls the states out
   from x0 and takes lam from the adjoint sweep.  width must equal
   bmpc_problem_output_width of every problem used.  Asynchronous. */
BMPC_API bmpc_status bmpc_batch_start_from_network(bmpc_batch* batch, const float* Y, int32_t rows,
                                                   int32_t width, void* stream);
/* Synchronise and copy the iteration history of problem i to hist (host,
   hist_cap x 6). */
BMPC_API bmpc_status bmpc_batch_history(bmpc_batch* batch, int32_t i, double* hist, void* stream);

/* ------------------------------------------------------------------------
 * Learned warm start.  The paper motivates the augmented Lagrangian by how
 * easily it is warm-started (Introduction; Sec. III); this library adds a
 * multilayer perceptron that maps a problem description to a starting
 * iterate.  Network: widths w_0 .. w_L; hidden layers
 *   A_{l+1} = gelu(A_l W_l + b_l),   gelu(z) = z/2 (1 + erf(z / sqrt 2)),
 * output Y = A_{L-1} W_{L-1} + b_{L-1} (linear).  Weights and activations
 * are BF16 (round to nearest even), every product accumulates in FP32 on the
 * matrix cores; master weights, gradients and Adam moments are FP32.
 * Parameter vector (FP32, host): W_0 .. W_{L-1} (each w_l x w_{l+1},
 * row-major), then b_0 .. b_{L-1}.  Loss: mean over all B * w_L outputs of
 * (Y - T)^2.  Device arrays X (B x w_0), Y and T (B x w_L) are row-major
 * FP32.  The network owns all its device memory; calls on one network must
 * not overlap.
 * ---------------------------------------------------------------------- */
typedef struct bmpc_mlp bmpc_mlp;
/* widths: host array of n_layers + 1 entries (each in [1, 65536]);
   n_layers in [1, 16]; max_batch >= 1 bounds B of every later call.
   Parameters start at zero.  BMPC_ERR_OOM if device memory runs out. */
BMPC_API bmpc_status bmpc_mlp_create(const int32_t* widths, int32_t n_layers, int32_t max_batch,
                                     bmpc_mlp** out);
BMPC_API void bmpc_mlp_destroy(bmpc_mlp* net);
/* Length of the parameter vector (0 for NULL). */
BMPC_API int64_t bmpc_mlp_num_params(const bmpc_mlp* net);
/* Load parameters (host FP32, synchronous) and reset the Adam state.
   BMPC_ERR_NONFINITE on a NaN/Inf entry. */
BMPC_API bmpc_status bmpc_mlp_set_params(bmpc_mlp* net, const float* params);
/* Input map applied in FP32 before the input is rounded to BF16:
   A_0 = bf16((X - shift) * scale) column by column (host arrays of w_0
   entries; synchronous).  Default shift 0, scale 1.  Lets a caller feed
   raw features whose mean is large against their spread. */
BMPC_API bmpc_status bmpc_mlp_set_input_map(bmpc_mlp* net, const float* shift, const float* scale);
/* Copy the FP32 master parameters to host (synchronous). */
BMPC_API bmpc_status bmpc_mlp_get_params(bmpc_mlp* net, float* params);
/* Inference: Y = network(X) for B rows, 1 <= B <= max_batch.  X is
   converted to BF16 first.  Asynchronous on `stream`. */
BMPC_API bmpc_status bmpc_mlp_forward(bmpc_mlp* net, const float* X, int32_t B, float* Y, void* stream);
/* Loss and its gradient with respect to the FP32 master parameters
   (evaluated through the BF16 copies); grad (host, num_params, nullable)
   and loss (host, nullable) are filled, then the call synchronises. */
BMPC_API bmpc_status bmpc_mlp_gradients(bmpc_mlp* net, const float* X, const float* T, int32_t B,
                                        float* grad, float* loss, void* stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, step
   size lr > 0) on the loss of (X, T); loss (host, nullable) receives the
   loss before the step and makes the call synchronous. */
BMPC_API bmpc_status bmpc_mlp_train_step(bmpc_mlp* net, const float* X, const float* T, int32_t B, float lr,
                                         float* loss, void* stream);
/* The network's matrix-core GEMM on its own: C (M x N, FP32, row-major) =
   op(A) op(B) with BF16 bit patterns A (M x K, or K x M when trans_a) and
   B (K x N, or N x K when trans_b), all device, row-major.  trans_a and
   trans_b together are BMPC_ERR_UNSUPPORTED.  Asynchronous. */
BMPC_API bmpc_status bmpc_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t trans_a,
                                    const uint16_t* B, int32_t trans_b, float* C, void* stream);

/* ------------------------------------------------------------------------
 * Launch configuration of batched solves and graph replay.
 * ---------------------------------------------------------------------- */
/* Autotuner: time every compiled (backward variant, threads per problem)
   pair on this batch (reps solves each, with settings s and warm bits warm,
   each from the batch's current state) and keep the one with the shortest
   time per inner iteration (launch time divided by the inner iterations
   summed over the batch) for launches with riccati_variant =
   BMPC_RICCATI_AUTO and block_size = 0.  The batch state is restored
   afterwards; its stats and history are those of the last run.
   variant_out, block_out (host, nullable) receive the choice and ms_out
   (host, nullable, bmpc_batch_tune_candidates() entries) each candidate's
   time per inner iteration in ms.  Synchronous.  Different choices sum the
   merit and KKT reductions in different orders, so iterates can differ by
   rounding; the per-iteration time keeps such differences in iteration
   counts out of the choice. */
BMPC_API bmpc_status bmpc_batch_tune(bmpc_batch* batch, const bmpc_settings* s, int32_t warm, int32_t reps,
                                     int32_t* variant_out, int32_t* block_out, double* ms_out, void* stream);
/* Number of tuning candidates; fills up to cap of their (variant, block)
   pairs in tuning order (host arrays, nullable). */
BMPC_API int32_t bmpc_batch_tune_candidates(int32_t* variants, int32_t* blocks, int32_t cap);
/* Autotuner with a time budget and a cache keyed by the batch's shape
   (problem count, warm bits, and each problem's node, depth, leaf and
   segment counts).  cache_path (host string, nullable): a text file of
   lines "bmpc-autotune <key> <variant> <block> <ms per inner iteration>";
   if it holds the batch's key, that choice is kept without any timing run
   (*from_cache = 1).  Otherwise every candidate is timed once, then in
   further rounds while budget_ms of host time have not passed (at most 100
   runs each), the one with the shortest time per inner iteration is kept
   (as bmpc_batch_tune) and a line is appended to the cache.  variant_out,
   block_out, ms_per_iter_out, from_cache: host, nullable.  Synchronous;
   the batch state is restored.  A cache that cannot be appended to ->
   BMPC_ERR_INVALID_ARG (the choice is still kept). */
BMPC_API bmpc_status bmpc_batch_autotune(bmpc_batch* batch, const bmpc_settings* s, int32_t warm,
                                         int32_t budget_ms, const char* cache_path, int32_t* variant_out,
                                         int32_t* block_out, double* ms_per_iter_out, int32_t* from_cache,
                                         void* stream);

/* Graph capture of asynchronous library calls on a created (non-default)
   stream: bmpc_graph_begin(stream), then any of bmpc_batch_launch,
   bmpc_batch_shift, bmpc_batch_start_from_network, bmpc_batch_state,
   bmpc_mlp_forward, bmpc_lqr_solve on that stream, then
   bmpc_graph_end(stream, &graph).  Synchronous calls (stats, history,
   tuning, *_create) fail inside a capture.  bmpc_graph_launch replays the
   whole sequence with the arguments it was recorded with (same buffers,
   same settings).  Kernel timing skips launches inside a capture. */
typedef struct bmpc_graph bmpc_graph;
BMPC_API bmpc_status bmpc_graph_begin(void* stream);
BMPC_API bmpc_status bmpc_graph_end(void* stream, bmpc_graph** out);
BMPC_API bmpc_status bmpc_graph_launch(bmpc_graph* graph, void* stream);
BMPC_API void bmpc_graph_destroy(bmpc_graph* graph);

/* ------------------------------------------------------------------------
 * Kernel timing.  When enabled, every kernel launch of the library is
 * bracketed by a pair of HIP events recorded on its own stream (this adds a
 * small gap between launches).
 * ---------------------------------------------------------------------- */
/* Enable (on != 0) or disable timing; clears the accumulated totals. */
BMPC_API bmpc_status bmpc_profile_enable(int32_t on);
/* Restrict timing to the launches whose kernel name equals `name` (host
   string, copied; NULL or "" times every launch again), so that a run can
   time its dominant kernel without the event gaps around the others. */
BMPC_API bmpc_status bmpc_profile_only(const char* name);
/* Waits for the recorded events and returns the number of distinct kernel
   names timed since the last read; fills up to `cap` entries: names
   (host, 64 bytes per entry, NUL-terminated), total_ms (host, summed event
   time) and launches (host, launch count).  Clears the totals.  Any output
   pointer may be NULL. */
BMPC_API int32_t bmpc_profile_read(char* names, double* total_ms, int32_t* launches, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* BMPC_H */
