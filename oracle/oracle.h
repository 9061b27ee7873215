/*
 * CPU FP64 oracle for the branch-MPC hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code with the HIP library and includes nothing
 * from it.  Everything here is plain, serial, double-precision C written
 * for readability, not speed.
 *
 * Array conventions (oracle only): node-major, row-major matrices, i.e.
 * A[i*nx*nx + r*nx + c] is entry (r, c) of the matrix of node i.
 * Tree: parent[0] = -1 and 0 <= parent[i] < i for i >= 1.
 * Edge-indexed dynamics: (A_i, B_i, c_i) stored at node i describe the
 * transition from parent(i) into i:  x_i = A_i x_p + B_i u_p + c_i.
 */
#ifndef BMPC_ORACLE_H
#define BMPC_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_ERR_INVALID_ARG = 1,
    ORC_ERR_TOPOLOGY = 2,
    ORC_ERR_NOT_PD = 3,
    ORC_ERR_NONFINITE = 4,
    ORC_ERR_MAXITER = 5,
    ORC_ERR_LINESEARCH = 6
};

/* ---- tree LQR (serial tree Riccati), oracle_lqr.c ---------------------- */
int orc_tree_lqr(int N, int nx, int nu, const int* parent,
                 const double* A, const double* B, const double* c,
                 const double* Q, const double* R, const double* M,
                 const double* q, const double* r, const double* x0,
                 double* x, double* u, double* lam,
                 double* K, double* k, double* P, double* p, int* bad_node);
/* The same recursion carried out in long double (x87 extended precision);
 * inputs and outputs are double.  Reference for badly conditioned problems. */
int orc_tree_lqr_ld(int N, int nx, int nu, const int* parent,
                    const double* A, const double* B, const double* c,
                    const double* Q, const double* R, const double* M,
                    const double* q, const double* r, const double* x0,
                    double* x, double* u, double* lam,
                    double* K, double* k, double* P, double* p, int* bad_node);
/* The same recursion in single precision (inputs rounded to float, outputs
 * widened to double): the FP32 variant of the solver, serially. */
int orc_tree_lqr_f(int N, int nx, int nu, const int* parent,
                   const double* A, const double* B, const double* c,
                   const double* Q, const double* R, const double* M,
                   const double* q, const double* r, const double* x0,
                   double* x, double* u, double* lam,
                   double* K, double* k, double* P, double* p, int* bad_node);

/* ---- branch-MPC problem and AL multiple-shooting iLQR, oracle_bmpc.c ---- */
#define ORC_NX 4
#define ORC_NU 2
#define ORC_NG 5 /* constraint slots per node: 4 input bounds + 1 obstacle */

typedef struct {
    int model;          /* 0 = kinematic bicycle (RK4), 1 = linear x+ = Al x + Bl u */
    double wheelbase;   /* bicycle wheelbase L */
    double dt;          /* step */
    double Qd[4];       /* diagonal state weight */
    double Rd[2];       /* diagonal input weight */
    double a_max;       /* |u0| <= a_max */
    double steer_max;   /* |u1| <= steer_max */
    double obs_r;       /* obstacle radius */
    double Al[16];      /* linear model only */
    double Bl[8];       /* linear model only */
} orc_model;

typedef struct {
    int N;
    const int* parent;
    const double* weight;    /* (N) node probability weight pi_n */
    const double* ref;       /* (N,4) node reference */
    const double* obs;       /* (N,2) obstacle centre used by node n */
    const int* has_obs;      /* (N) 1 if node n carries the obstacle constraint */
    const double* x0;        /* (4) */
    orc_model model;
} orc_problem;

typedef struct {
    double eps_tol, tau, omega0, eta0, a_omega, b_omega, a_eta, b_eta;
    double rho0, mu0, armijo_beta;
    int n_alpha, max_outer, max_inner, max_ls_fail;
    int max_iter_total; /* cap on inner iterations over all outer ones, 0 = none */
    int ls_rounds;      /* backtracking rounds of n_alpha step sizes each */
    int hessian;        /* 0 = Gauss-Newton, 1 = exact with eigenvalue modification */
    double eig_floor;   /* exact node Hessian: eigenvalues raised to at least
                           eig_floor * max(1, largest |eigenvalue| of the block) */
} orc_settings;

typedef struct {
    int status, outer_it, inner_it, ls_failures, bad_node, start;
    double r_kkt, viol, rho, mu, merit;
} orc_stats;

void orc_settings_default(orc_settings* s);

/* warm bits: 1 = x,u supplied, 2 = lam supplied, 4 = ye supplied (clamped at
   zero), 8 = u supplied with x from the rollout, 16 = keep the cold start
   instead if its max(KKT residual, violation) is smaller */
int orc_bmpc_solve(const orc_problem* pb, const orc_settings* st, int warm,
                   double* x, double* u, double* lam, double* ye,
                   orc_stats* stats, double* hist, int hist_cap);

/* pieces exported for pinning */
void orc_rk4(const orc_model* m, const double* x, const double* u, double* xn,
             double* A, double* B);
/* ---- exact Hessian pieces, oracle_hess.c ---- */
/* H (6 x 6, z = (x, u)) = second derivatives of mu^T F(x, u), F the model's
 * step (zero for the linear model). */
void orc_rk4_hessian(const orc_model* m, const double* x, const double* u, const double* mu,
                     double* H);
/* Symmetric eigendecomposition A = V diag(w) V^T (n <= 6, cyclic Jacobi);
 * V row-major, eigenvector k in column k. */
int orc_sym_eig(int n, const double* A, double* w, double* V);
/* out = V diag(max(w, delta)) V^T */
int orc_eig_modify(int n, const double* A, double delta, double* out);
/* Quadratic model of node n (all state arrays of the whole tree): q, r and
 * the Hessian blocks Q (4x4), R (2x2), M (2x4) for the given Hessian choice;
 * modify = 0 leaves the exact Hessian unmodified (for the pins). */
void orc_node_quadratic(const orc_problem* pb, int n, const double* x, const double* u,
                        const double* lam, const double* ye, double rho, int hessian, double delta,
                        int modify, double* q, double* r, double* Q, double* R, double* M);
void orc_node_weights(int N, const int* parent, const double* leaf_prob, double* weight);
void orc_node_refs(int N, const int* parent, const double* leaf_prob, const double* leaf_offset,
                   double dt, double speed, double* ref);
double orc_node_terms(const orc_problem* pb, int n, const double* x, const double* u,
                      const double* ye, double rho, double* g, double* gx, double* gu,
                      double* Hxx, double* Huu);
double orc_augmented_lagrangian(const orc_problem* pb, const double* x, const double* u,
                                const double* ye, double rho);
double orc_merit(const orc_problem* pb, const double* x, const double* u, const double* lam,
                 const double* ye, double rho, double mu);
double orc_kkt(const orc_problem* pb, const double* x, const double* u, const double* lam,
               const double* ye, double rho);
/* One search direction and the slope of the merit along it: the tree LQR
 * step (dx, du, lh) at the given point, then with J_d dz = -d,
 *   out[0] = g^T dz, out[1] = dz^T H dz, out[2] = (lh - 2 lam)^T d,
 *   out[3] = d^T d, out[4] = mu_hat (0 if d = 0), out[5] = mu after the
 *   update, out[6] = phi'(0) at that mu, out[7] = phi(0) at that mu.
 * Returns the LQR status. */
int orc_direction_h(const orc_problem* pb, const double* x, const double* u, const double* lam,
                    const double* ye, double rho, double mu, int hessian, double delta, double* dx,
                    double* du, double* lh, double* out);
int orc_direction(const orc_problem* pb, const double* x, const double* u, const double* lam,
                  const double* ye, double rho, double mu, double* dx, double* du, double* lh,
                  double* out);
double orc_violation(const orc_problem* pb, const double* x, const double* u,
                     const double* ye, double rho);
void orc_adjoint(const orc_problem* pb, const double* x, const double* u,
                 const double* ye, double rho, double* lam);
void orc_rollout(const orc_problem* pb, const double* u, double* x);
void orc_shift(const orc_problem* pb, const double* x, const double* u, const double* lam,
               const double* ye, const double* x0_meas, double* ref_new, double* x0_new, double* xs,
               double* us, double* lams, double* yes);

/* ---- warm-start network, oracle_mlp.c ---------------------------------- */
double orc_bf16(double x);
double orc_gelu(double z);
double orc_gelu_prime(double z);
int orc_mlp_forward(int L, const int* w, int B, const double* params, const double* X, int quant, double* Y);
int orc_mlp_backward(int L, const int* w, int B, const double* params, const double* X, const double* T,
                     int quant, double* grad, double* loss);
void orc_adam(long n, double* p, const double* g, double* m, double* v, int t, double lr, double b1, double b2,
              double eps);

#ifdef __cplusplus
}
#endif
#endif
