/*
 * Oracle: branch-MPC problem on a trajectory tree and the augmented-
 * Lagrangian multiple-shooting iLQR that solves it.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Problem (Sec. II-B, eq. bmpc): minimise the sum of node costs over the
 * state and input trees subject to the tree dynamics x_j = f(x_p, u_p) and
 * per-node inequality constraints g_n <= 0.  The workload is a kinematic
 * bicycle; the constraint set is four input bounds at control nodes and one
 * round obstacle per node of an obstacle-bearing segment.
 *
 * Readings of the paper taken here (each stated where it is used):
 *   - node weights pi_n multiply the stage and terminal costs, not the
 *     constraints; pi_n is the total probability of the scenarios through n;
 *   - Hessian: Gauss-Newton (dynamics and constraint curvature dropped) by
 *     default; or the exact Hessian of the Lagrangian per node with its
 *     eigenvalues raised to at least delta times the block's largest
 *     |eigenvalue| (at least 1) (settings.hessian = 1);
 *   - the merit's J is the augmented objective L_a; lambda is line-searched
 *     jointly with (x, u) towards the LQR costates;
 *   - alpha set {2^0 .. 2^-(K-1)}, Armijo constant 1e-4;
 *   - outer-loop tolerances are divided by powers of rho (rho > 1 here) and
 *     the multiplier update is the standard PHR step y <- max(0, y + rho g).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define NX ORC_NX
#define NU ORC_NU
#define NG ORC_NG
#define HALF_PI 1.5707963267948966

void orc_settings_default(orc_settings* s)
{
    s->eps_tol = 1e-6;
    s->tau = 100.0;
    s->omega0 = 1.0;
    s->eta0 = 0.1;
    s->a_omega = 1.0;
    s->b_omega = 1.0;
    s->a_eta = 0.1;
    s->b_eta = 0.9;
    s->rho0 = 100.0;
    s->mu0 = 100.0;
    s->armijo_beta = 1e-4;
    s->n_alpha = 10;
    s->max_outer = 50;
    s->max_inner = 100;
    s->max_ls_fail = 3;
    s->max_iter_total = 0;
    s->ls_rounds = 3;
    s->hessian = 0;
    s->eig_floor = 1e-9;
}

/* ------------------------------------------------------------------------
 * Dynamics.  Bicycle: continuous  d/dt [px,py,psi,v] =
 *   [v cos(psi), v sin(psi), v tan(delta)/L, a],  u = [a, delta],
 * discretised with one classical RK4 step of length dt (input held).
 * Jacobians follow the RK4 stages by the chain rule.
 * ---------------------------------------------------------------------- */
static void bicycle_ct(double L, const double* x, const double* u, double* f,
                       double* Jx, double* Ju)
{
    const double c = cos(x[2]), s = sin(x[2]);
    const double v = x[3];
    const double td = tan(u[1]);
    const double cd = cos(u[1]);
    f[0] = v * c;
    f[1] = v * s;
    f[2] = v * td / L;
    f[3] = u[0];
    memset(Jx, 0, sizeof(double) * NX * NX);
    memset(Ju, 0, sizeof(double) * NX * NU);
    Jx[0 * NX + 2] = -v * s;
    Jx[0 * NX + 3] = c;
    Jx[1 * NX + 2] = v * c;
    Jx[1 * NX + 3] = s;
    Jx[2 * NX + 3] = td / L;
    Ju[2 * NU + 1] = v / (L * cd * cd);
    Ju[3 * NU + 0] = 1.0;
}

void orc_rk4(const orc_model* m, const double* x, const double* u, double* xn,
             double* A, double* B)
{
    if (m->model == 1) {
        for (int a = 0; a < NX; ++a) {
            double t = 0.0;
            for (int b = 0; b < NX; ++b) t += m->Al[a * NX + b] * x[b];
            for (int b = 0; b < NU; ++b) t += m->Bl[a * NU + b] * u[b];
            xn[a] = t;
        }
        if (A) memcpy(A, m->Al, sizeof(double) * NX * NX);
        if (B) memcpy(B, m->Bl, sizeof(double) * NX * NU);
        return;
    }
    const double h = m->dt, L = m->wheelbase;
    double k[4][NX], dkx[4][NX * NX], dku[4][NX * NU];
    double Jx[NX * NX], Ju[NX * NU];
    double X[NX], dXx[NX * NX], dXu[NX * NU];
    static const double stage_c[4] = {0.0, 0.5, 0.5, 1.0};
    for (int st = 0; st < 4; ++st) {
        /* stage point X = x + c h k_{st-1} and its derivatives */
        for (int a = 0; a < NX; ++a) {
            X[a] = x[a] + (st ? stage_c[st] * h * k[st - 1][a] : 0.0);
            for (int b = 0; b < NX; ++b)
                dXx[a * NX + b] = (a == b ? 1.0 : 0.0) +
                                  (st ? stage_c[st] * h * dkx[st - 1][a * NX + b] : 0.0);
            for (int b = 0; b < NU; ++b)
                dXu[a * NU + b] = st ? stage_c[st] * h * dku[st - 1][a * NU + b] : 0.0;
        }
        bicycle_ct(L, X, u, k[st], Jx, Ju);
        for (int a = 0; a < NX; ++a) {
            for (int b = 0; b < NX; ++b) {
                double t = 0.0;
                for (int l = 0; l < NX; ++l) t += Jx[a * NX + l] * dXx[l * NX + b];
                dkx[st][a * NX + b] = t;
            }
            for (int b = 0; b < NU; ++b) {
                double t = Ju[a * NU + b];
                for (int l = 0; l < NX; ++l) t += Jx[a * NX + l] * dXu[l * NU + b];
                dku[st][a * NU + b] = t;
            }
        }
    }
    for (int a = 0; a < NX; ++a)
        xn[a] = x[a] + h / 6.0 * (k[0][a] + 2.0 * k[1][a] + 2.0 * k[2][a] + k[3][a]);
    if (A)
        for (int e = 0; e < NX * NX; ++e)
            A[e] = ((e / NX) == (e % NX) ? 1.0 : 0.0) +
                   h / 6.0 * (dkx[0][e] + 2.0 * dkx[1][e] + 2.0 * dkx[2][e] + dkx[3][e]);
    if (B)
        for (int e = 0; e < NX * NU; ++e)
            B[e] = h / 6.0 * (dku[0][e] + 2.0 * dku[1][e] + 2.0 * dku[2][e] + dku[3][e]);
}

/* ------------------------------------------------------------------------
 * Scenario data -> node data.
 * pi_n = sum of the probabilities of the leaves below n.  The reference of
 * node n at stage t is [speed*t*dt, ybar_n, 0, speed] where ybar_n is the
 * pi-weighted mean lateral offset of the scenarios through n (the weighted
 * sum of the scenario tracking costs equals pi_n times the tracking cost
 * about this mean, up to a constant).
 * ---------------------------------------------------------------------- */
static int* leaf_index_map(int N, const int* parent)
{
    int* nch = calloc((size_t)N, sizeof(int));
    for (int i = 1; i < N; ++i) nch[parent[i]]++;
    int* idx = malloc(sizeof(int) * (size_t)N);
    int z = 0;
    for (int i = 0; i < N; ++i) idx[i] = nch[i] == 0 ? z++ : -1;
    free(nch);
    return idx;
}

void orc_node_weights(int N, const int* parent, const double* leaf_prob, double* weight)
{
    int* li = leaf_index_map(N, parent);
    for (int i = 0; i < N; ++i) weight[i] = li[i] >= 0 ? leaf_prob[li[i]] : 0.0;
    for (int i = N - 1; i >= 1; --i) weight[parent[i]] += weight[i];
    free(li);
}

void orc_node_refs(int N, const int* parent, const double* leaf_prob, const double* leaf_offset,
                   double dt, double speed, double* ref)
{
    int* li = leaf_index_map(N, parent);
    double* w = calloc((size_t)N, sizeof(double));
    double* wy = calloc((size_t)N, sizeof(double));
    int* stage = calloc((size_t)N, sizeof(int));
    for (int i = 1; i < N; ++i) stage[i] = stage[parent[i]] + 1;
    for (int i = 0; i < N; ++i)
        if (li[i] >= 0) {
            w[i] = leaf_prob[li[i]];
            wy[i] = leaf_prob[li[i]] * leaf_offset[li[i]];
        }
    for (int i = N - 1; i >= 1; --i) {
        w[parent[i]] += w[i];
        wy[parent[i]] += wy[i];
    }
    for (int i = 0; i < N; ++i) {
        ref[i * 4 + 0] = speed * stage[i] * dt;
        ref[i * 4 + 1] = w[i] > 0.0 ? wy[i] / w[i] : 0.0;
        ref[i * 4 + 2] = 0.0;
        ref[i * 4 + 3] = speed;
    }
    free(li); free(w); free(wy); free(stage);
}

/* ------------------------------------------------------------------------
 * Node terms of the augmented objective (eq. AL):
 *   L_a,n = pi_n * stage cost + rho/2 || max(0, g_n + y_n/rho) ||^2
 * Returns L_a,n and fills g (NG slots; inactive slots -> -inf), the exact
 * gradients gx, gu, and the Gauss-Newton Hessian blocks Hxx, Huu (the
 * cross block is zero: no constraint mixes x and u).  Any output may be NULL.
 * Slot layout: 0: u0 - a_max, 1: -u0 - a_max, 2: u1 - steer_max,
 * 3: -u1 - steer_max (control nodes only), 4: obs_r - |p - o| with p the
 * position (px, py) and o the obstacle centre, i.e. the distance must exceed
 * the radius (nodes of obstacle-bearing segments; at |p - o| = 0 the
 * gradient direction -e_x is used).  Active set for the Hessian:
 * g + y/rho > 0.
 * ---------------------------------------------------------------------- */
static int is_leaf_tab(const orc_problem* pb, int n, const int* nch)
{
    (void)pb;
    return nch[n] == 0;
}

static double node_terms_impl(const orc_problem* pb, int n, int leaf, const double* x,
                              const double* u, const double* ye, double rho, double* g,
                              double* gx, double* gu, double* Hxx, double* Huu)
{
    const orc_model* m = &pb->model;
    const double w = pb->weight[n];
    const double* rf = pb->ref + (size_t)n * 4;
    double val = 0.0;
    double lg[NG], lgx[NX], lgu[NU], lHxx[NX * NX], lHuu[NU * NU];
    memset(lgx, 0, sizeof lgx);
    memset(lgu, 0, sizeof lgu);
    memset(lHxx, 0, sizeof lHxx);
    memset(lHuu, 0, sizeof lHuu);
    for (int a = 0; a < NX; ++a) {
        const double e = x[a] - rf[a];
        val += 0.5 * w * m->Qd[a] * e * e;
        lgx[a] = w * m->Qd[a] * e;
        lHxx[a * NX + a] = w * m->Qd[a];
    }
    if (!leaf)
        for (int a = 0; a < NU; ++a) {
            val += 0.5 * w * m->Rd[a] * u[a] * u[a];
            lgu[a] = w * m->Rd[a] * u[a];
            lHuu[a * NU + a] = w * m->Rd[a];
        }
    for (int s = 0; s < NG; ++s) lg[s] = -INFINITY;
    if (!leaf) {
        lg[0] = u[0] - m->a_max;
        lg[1] = -u[0] - m->a_max;
        lg[2] = u[1] - m->steer_max;
        lg[3] = -u[1] - m->steer_max;
        for (int s = 0; s < 4; ++s) {
            const double t = lg[s] + ye[s] / rho;
            if (t > 0.0) {
                const int a = s / 2;
                const double sg = (s % 2 == 0) ? 1.0 : -1.0;
                val += 0.5 * rho * t * t;
                lgu[a] += rho * t * sg;
                lHuu[a * NU + a] += rho;
            }
        }
    }
    if (pb->has_obs[n]) {
        const double dx = x[0] - pb->obs[n * 2 + 0];
        const double dy = x[1] - pb->obs[n * 2 + 1];
        const double dist = sqrt(dx * dx + dy * dy);
        lg[4] = m->obs_r - dist;
        const double t = lg[4] + ye[4] / rho;
        if (t > 0.0) {
            const double j0 = dist > 0.0 ? -dx / dist : -1.0, j1 = dist > 0.0 ? -dy / dist : 0.0;
            val += 0.5 * rho * t * t;
            lgx[0] += rho * t * j0;
            lgx[1] += rho * t * j1;
            lHxx[0 * NX + 0] += rho * j0 * j0;
            lHxx[0 * NX + 1] += rho * j0 * j1;
            lHxx[1 * NX + 0] += rho * j1 * j0;
            lHxx[1 * NX + 1] += rho * j1 * j1;
        }
    }
    if (g) memcpy(g, lg, sizeof lg);
    if (gx) memcpy(gx, lgx, sizeof lgx);
    if (gu) memcpy(gu, lgu, sizeof lgu);
    if (Hxx) memcpy(Hxx, lHxx, sizeof lHxx);
    if (Huu) memcpy(Huu, lHuu, sizeof lHuu);
    return val;
}

static int* child_counts(const orc_problem* pb)
{
    int* nch = calloc((size_t)pb->N, sizeof(int));
    for (int i = 1; i < pb->N; ++i) nch[pb->parent[i]]++;
    return nch;
}

/* The quadratic model of node n (Sec. IV-A, search direction): gradient
 * (q, r) of the augmented objective and the Hessian blocks Q, R, M of the
 * node's part of the Lagrangian
 *   L_a,n(x_n, u_n) + sum_{j child of n} lam_j^T f(x_n, u_n).
 * hessian = 0: Gauss-Newton (M = 0).  hessian = 1: exact, i.e. in addition
 *   - the curvature of the active obstacle penalty, rho t grad^2 g with
 *     t = g + y/rho and grad^2 g = -(I - e e^T) / dist (e the unit vector
 *     from the obstacle to the position), and
 *   - the dynamics curvature sum_a mu_a grad^2 F_a, mu = sum of the
 *     children's multipliers;
 * then, with modify, the whole (x, u) block (x only at a leaf) has its
 * eigenvalues below delta * max(1, largest |eigenvalue|) raised to that
 * floor. */
static void node_quadratic(const orc_problem* pb, const int* nch, int n, const double* x,
                           const double* u, const double* lam, const double* ye, double rho,
                           int hessian, double delta, int modify, double* q, double* r, double* Q,
                           double* R, double* M)
{
    const int leaf = nch[n] == 0;
    const double* xn = x + (size_t)n * NX;
    const double* un = u + (size_t)n * NU;
    const double* yn = ye + (size_t)n * NG;
    double Hxx[NX * NX], Huu[NU * NU];
    node_terms_impl(pb, n, leaf, xn, un, yn, rho, NULL, q, r, Hxx, Huu);
    memcpy(Q, Hxx, sizeof Hxx);
    memcpy(R, Huu, sizeof Huu);
    memset(M, 0, sizeof(double) * NU * NX);
    if (hessian == 0) return;
    enum { NZ = NX + NU };
    double H[NZ * NZ];
    memset(H, 0, sizeof H);
    for (int a = 0; a < NX; ++a)
        for (int b = 0; b < NX; ++b) H[a * NZ + b] = Hxx[a * NX + b];
    for (int a = 0; a < NU; ++a)
        for (int b = 0; b < NU; ++b) H[(NX + a) * NZ + NX + b] = Huu[a * NU + b];
    if (pb->has_obs[n]) {
        const double ddx = xn[0] - pb->obs[n * 2 + 0];
        const double ddy = xn[1] - pb->obs[n * 2 + 1];
        const double dist = sqrt(ddx * ddx + ddy * ddy);
        const double t = (pb->model.obs_r - dist) + yn[4] / rho;
        if (t > 0.0 && dist > 0.0) {
            const double e[2] = {ddx / dist, ddy / dist};
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b)
                    H[a * NZ + b] += rho * t * (-((a == b ? 1.0 : 0.0) - e[a] * e[b]) / dist);
        }
    }
    if (!leaf) {
        double mu[NX] = {0, 0, 0, 0}, Hd[NZ * NZ];
        for (int j = 1; j < pb->N; ++j)
            if (pb->parent[j] == n)
                for (int a = 0; a < NX; ++a) mu[a] += lam[(size_t)j * NX + a];
        orc_rk4_hessian(&pb->model, xn, un, mu, Hd);
        for (int e = 0; e < NZ * NZ; ++e) H[e] += Hd[e];
    }
    const int nz = leaf ? NX : NZ;
    double Hm[NZ * NZ], Hs[NZ * NZ];
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < nz; ++b) Hs[a * nz + b] = H[a * NZ + b];
    if (modify) {
        /* floor relative to the block's largest |eigenvalue| (at least 1) */
        double w[NZ], V[NZ * NZ], big = 1.0;
        orc_sym_eig(nz, Hs, w, V);
        for (int i = 0; i < nz; ++i) big = fmax(big, fabs(w[i]));
        orc_eig_modify(nz, Hs, delta * big, Hm);
    } else
        memcpy(Hm, Hs, sizeof(double) * nz * nz);
    for (int a = 0; a < NX; ++a)
        for (int b = 0; b < NX; ++b) Q[a * NX + b] = Hm[a * nz + b];
    if (!leaf) {
        for (int a = 0; a < NU; ++a) {
            for (int b = 0; b < NX; ++b) M[a * NX + b] = Hm[(NX + a) * nz + b];
            for (int b = 0; b < NU; ++b) R[a * NU + b] = Hm[(NX + a) * nz + NX + b];
        }
    }
}

void orc_node_quadratic(const orc_problem* pb, int n, const double* x, const double* u,
                        const double* lam, const double* ye, double rho, int hessian, double delta,
                        int modify, double* q, double* r, double* Q, double* R, double* M)
{
    int* nch = child_counts(pb);
    node_quadratic(pb, nch, n, x, u, lam, ye, rho, hessian, delta, modify, q, r, Q, R, M);
    free(nch);
}

double orc_node_terms(const orc_problem* pb, int n, const double* x, const double* u,
                      const double* ye, double rho, double* g, double* gx, double* gu,
                      double* Hxx, double* Huu)
{
    int* nch = child_counts(pb);
    const int leaf = is_leaf_tab(pb, n, nch);
    free(nch);
    return node_terms_impl(pb, n, leaf, x, u, ye, rho, g, gx, gu, Hxx, Huu);
}

static double aug_lag(const orc_problem* pb, const int* nch, const double* x, const double* u,
                      const double* ye, double rho)
{
    double v = 0.0;
    for (int n = 0; n < pb->N; ++n)
        v += node_terms_impl(pb, n, nch[n] == 0, x + n * NX, u + n * NU, ye + n * NG, rho,
                             NULL, NULL, NULL, NULL, NULL);
    return v;
}

double orc_augmented_lagrangian(const orc_problem* pb, const double* x, const double* u,
                                const double* ye, double rho)
{
    int* nch = child_counts(pb);
    const double v = aug_lag(pb, nch, x, u, ye, rho);
    free(nch);
    return v;
}

/* defect of edge j: d_j = f(x_p, u_p) - x_j */
static void defect(const orc_problem* pb, int j, const double* x, const double* u, double* d,
                   double* A, double* B)
{
    const int p = pb->parent[j];
    double xn[NX];
    orc_rk4(&pb->model, x + p * NX, u + p * NU, xn, A, B);
    for (int a = 0; a < NX; ++a) d[a] = xn[a] - x[j * NX + a];
}

/* Merit of eq. merit with J := L_a:  phi = L_a + lam^T d + mu/2 d^T d */
/* The kinematic bicycle is defined for steering angles inside (-pi/2, pi/2):
 * tan has its pole at pi/2 and past it the yaw rate changes sign.  A trial
 * point outside that domain is not a point of the problem; its merit is +inf,
 * so the sufficient-decrease test rejects it and the search backtracks. */
static int in_model_domain(const orc_problem* pb, const int* nch, const double* u)
{
    if (pb->model.model != 0) return 1;
    for (int n = 0; n < pb->N; ++n)
        if (nch[n] > 0 && !(fabs(u[n * NU + 1]) < HALF_PI)) return 0;
    return 1;
}

static double merit_impl(const orc_problem* pb, const int* nch, const double* x,
                         const double* u, const double* lam, const double* ye, double rho,
                         double mu)
{
    if (!in_model_domain(pb, nch, u)) return INFINITY;
    double v = aug_lag(pb, nch, x, u, ye, rho);
    double ld = 0.0, dd = 0.0;
    for (int j = 1; j < pb->N; ++j) {
        double d[NX];
        defect(pb, j, x, u, d, NULL, NULL);
        for (int a = 0; a < NX; ++a) {
            ld += lam[j * NX + a] * d[a];
            dd += d[a] * d[a];
        }
    }
    return v + ld + 0.5 * mu * dd;
}

double orc_merit(const orc_problem* pb, const double* x, const double* u, const double* lam,
                 const double* ye, double rho, double mu)
{
    int* nch = child_counts(pb);
    const double v = merit_impl(pb, nch, x, u, lam, ye, rho, mu);
    free(nch);
    return v;
}

/* KKT residual of the relaxed problem (Sec. IV-A, inner stopping rule):
 *   grad_{x_j} = dL_a/dx_j - lam_j + sum_{c in ch(j)} A_c^T lam_c   (j != 0)
 *   grad_{u_n} = dL_a/du_n + sum_{c in ch(n)} B_c^T lam_c
 *   grad_lam   = d
 * r_kkt = max of the infinity norms. */
double orc_kkt(const orc_problem* pb, const double* x, const double* u, const double* lam,
               const double* ye, double rho)
{
    const int N = pb->N;
    int* nch = child_counts(pb);
    double* gxs = calloc((size_t)N * NX, sizeof(double));
    double* gus = calloc((size_t)N * NU, sizeof(double));
    double r = 0.0;
    for (int n = 0; n < N; ++n)
        node_terms_impl(pb, n, nch[n] == 0, x + n * NX, u + n * NU, ye + n * NG, rho, NULL,
                        gxs + n * NX, gus + n * NU, NULL, NULL);
    for (int j = 1; j < N; ++j) {
        double d[NX], A[NX * NX], B[NX * NU];
        const int p = pb->parent[j];
        defect(pb, j, x, u, d, A, B);
        for (int a = 0; a < NX; ++a) {
            if (fabs(d[a]) > r || isnan(d[a])) r = isnan(d[a]) ? NAN : fmax(r, fabs(d[a]));
            double t = 0.0;
            for (int b = 0; b < NX; ++b) t += A[b * NX + a] * lam[j * NX + b];
            gxs[p * NX + a] += t;
        }
        for (int a = 0; a < NU; ++a) {
            double t = 0.0;
            for (int b = 0; b < NX; ++b) t += B[b * NU + a] * lam[j * NX + b];
            gus[p * NU + a] += t;
        }
    }
    for (int n = 0; n < N && !isnan(r); ++n) {
        if (n != 0)
            for (int a = 0; a < NX; ++a) {
                const double v = gxs[n * NX + a] - lam[n * NX + a];
                if (isnan(v)) r = NAN;
                else r = fmax(r, fabs(v));
            }
        if (nch[n] > 0)
            for (int a = 0; a < NU; ++a) {
                const double v = gus[n * NU + a];
                if (isnan(v)) r = NAN;
                else r = fmax(r, fabs(v));
            }
    }
    free(nch); free(gxs); free(gus);
    return r;
}

/* Constraint violation c = || max(g, -y/rho) ||_inf over the active slots. */
double orc_violation(const orc_problem* pb, const double* x, const double* u,
                     const double* ye, double rho)
{
    int* nch = child_counts(pb);
    double c = 0.0;
    for (int n = 0; n < pb->N; ++n) {
        double g[NG];
        node_terms_impl(pb, n, nch[n] == 0, x + n * NX, u + n * NU, ye + n * NG, rho, g, NULL,
                        NULL, NULL, NULL);
        for (int s = 0; s < NG; ++s) {
            if (g[s] == -INFINITY) continue;
            c = fmax(c, fabs(fmax(g[s], -ye[n * NG + s] / rho)));
        }
    }
    free(nch);
    return c;
}

/* Adjoint sweep: lam_leaf = dL_a/dx, lam_j = dL_a/dx_j + sum_c A_c^T lam_c.
 * It makes grad_x of the Lagrangian vanish at the given point. */
void orc_adjoint(const orc_problem* pb, const double* x, const double* u, const double* ye,
                 double rho, double* lam)
{
    const int N = pb->N;
    int* nch = child_counts(pb);
    for (int n = 0; n < N; ++n)
        node_terms_impl(pb, n, nch[n] == 0, x + n * NX, u + n * NU, ye + n * NG, rho, NULL,
                        lam + n * NX, NULL, NULL, NULL);
    for (int j = N - 1; j >= 1; --j) {
        double d[NX], A[NX * NX];
        const int p = pb->parent[j];
        defect(pb, j, x, u, d, A, NULL);
        for (int a = 0; a < NX; ++a) {
            double t = 0.0;
            for (int b = 0; b < NX; ++b) t += A[b * NX + a] * lam[j * NX + b];
            lam[p * NX + a] += t;
        }
    }
    free(nch);
}

void orc_rollout(const orc_problem* pb, const double* u, double* x)
{
    memcpy(x, pb->x0, sizeof(double) * NX);
    for (int j = 1; j < pb->N; ++j)
        orc_rk4(&pb->model, x + pb->parent[j] * NX, u + pb->parent[j] * NU, x + j * NX, NULL,
                NULL);
}

/* Start point.  warm bits: 1 = x, u given; 8 = u given and x from the
 * exact rollout; 4 = ye given (negative entries set to zero); 2 = lam given,
 * otherwise lam from the adjoint sweep.  No bit: u = 0 and the rollout. */
static void start_point(const orc_problem* pb, const int* nch, int warm, double* x, double* u,
                        double* lam, double* ye, double rho)
{
    const int N = pb->N;
    if (!(warm & (1 | 8))) memset(u, 0, sizeof(double) * (size_t)N * NU);
    for (int n = 0; n < N; ++n)
        if (nch[n] == 0) memset(u + n * NU, 0, sizeof(double) * NU);
    if ((warm & 8) || !(warm & 1)) orc_rollout(pb, u, x);
    memcpy(x, pb->x0, sizeof(double) * NX);
    for (int i = 0; i < N * NG; ++i) ye[i] = (warm & 4) ? (ye[i] > 0.0 ? ye[i] : 0.0) : 0.0;
    if (!(warm & 2)) orc_adjoint(pb, x, u, ye, rho, lam);
}

/* quality of a start point: max(KKT residual, violation), NaN counted as +inf */
static double start_measure(const orc_problem* pb, const double* x, const double* u, const double* lam,
                            const double* ye, double rho)
{
    const double k = orc_kkt(pb, x, u, lam, ye, rho);
    const double v = orc_violation(pb, x, u, ye, rho);
    if (isnan(k) || isnan(v)) return INFINITY;
    return k > v ? k : v;
}

/* Linearise the dynamics and quadratise L_a at (x, u) (Gauss-Newton, Sec.
 * IV-A), solve the tree LQR in the deviations with delta x_0 = 0, and form
 * the merit's slope along the step.  The step satisfies J_d dz = -d, so with
 * lambda(alpha) = lambda + alpha (lh - lambda),
 *   phi'(0) = g^T dz + (lh - lambda)^T d + lambda^T J_d dz + mu d^T J_d dz
 *           = g^T dz + (lh - 2 lambda)^T d - mu ||d||^2.
 * Adaptive mu (Gill et al., cited in Sec. IV-A): the slope must not exceed
 * -1/2 dz^T H dz; mu_hat is the mu at which it equals that bound, and a mu
 * below mu_hat is raised to max(mu_hat, 2 mu).  sl receives g^T dz, dz^T H dz,
 * (lh - 2 lambda)^T d, ||d||^2, mu_hat, the new mu, phi'(0) and phi(0). */
static int direction_step(const orc_problem* pb, const int* nch, const double* x,
                          const double* u, const double* lam, const double* ye, double rho,
                          double mu, int hessian, double delta, double* A, double* B, double* c,
                          double* Q, double* R,
                          double* M, double* q, double* r, double* dx, double* du, double* lh,
                          double* K, double* kk, double* P, double* p, int* bad, double* sl)
{
    const int N = pb->N;
    const double zero_x[NX] = {0, 0, 0, 0};
    for (int n = 0; n < N; ++n) {
        node_quadratic(pb, nch, n, x, u, lam, ye, rho, hessian, delta, 1, q + n * NX, r + n * NU,
                       Q + n * NX * NX, R + n * NU * NU, M + n * NU * NX);
        if (n > 0) defect(pb, n, x, u, c + n * NX, A + n * NX * NX, B + n * NX * NU);
    }
    const int lst = orc_tree_lqr(N, NX, NU, pb->parent, A, B, c, Q, R, M, q, r, zero_x, dx,
                                 du, lh, K, kk, P, p, bad);
    if (lst != ORC_OK) return lst;
    double gtd = 0.0, dhd = 0.0, ld = 0.0, dd = 0.0;
    for (int n = 0; n < N; ++n) {
        const double* Qn = Q + n * NX * NX;
        const double* Rn = R + n * NU * NU;
        const double* Mn = M + n * NU * NX;
        for (int a = 0; a < NX; ++a) {
            gtd += q[n * NX + a] * dx[n * NX + a];
            for (int b = 0; b < NX; ++b) dhd += dx[n * NX + a] * Qn[a * NX + b] * dx[n * NX + b];
        }
        if (nch[n] > 0)
            for (int a = 0; a < NU; ++a) {
                gtd += r[n * NU + a] * du[n * NU + a];
                for (int b = 0; b < NU; ++b) dhd += du[n * NU + a] * Rn[a * NU + b] * du[n * NU + b];
                for (int b = 0; b < NX; ++b) dhd += 2.0 * du[n * NU + a] * Mn[a * NX + b] * dx[n * NX + b];
            }
        if (n > 0)
            for (int a = 0; a < NX; ++a) {
                ld += (lh[n * NX + a] - 2.0 * lam[n * NX + a]) * c[n * NX + a];
                dd += c[n * NX + a] * c[n * NX + a];
            }
    }
    double mu_hat = 0.0;
    if (dd > 0.0) {
        mu_hat = (gtd + ld + 0.5 * dhd) / dd;
        if (mu < mu_hat) mu = fmax(mu_hat, 2.0 * mu);
    }
    sl[0] = gtd;
    sl[1] = dhd;
    sl[2] = ld;
    sl[3] = dd;
    sl[4] = mu_hat;
    sl[5] = mu;
    sl[6] = gtd + ld - mu * dd;
    sl[7] = merit_impl(pb, nch, x, u, lam, ye, rho, mu);
    return ORC_OK;
}

int orc_direction(const orc_problem* pb, const double* x, const double* u, const double* lam,
                  const double* ye, double rho, double mu, double* dx, double* du, double* lh,
                  double* out)
{
    return orc_direction_h(pb, x, u, lam, ye, rho, mu, 0, 0.0, dx, du, lh, out);
}

int orc_direction_h(const orc_problem* pb, const double* x, const double* u, const double* lam,
                    const double* ye, double rho, double mu, int hessian, double delta, double* dx,
                    double* du, double* lh, double* out)
{
    const int N = pb->N;
    int* nch = child_counts(pb);
    double* A = calloc((size_t)N * NX * NX, sizeof(double));
    double* B = calloc((size_t)N * NX * NU, sizeof(double));
    double* c = calloc((size_t)N * NX, sizeof(double));
    double* Q = calloc((size_t)N * NX * NX, sizeof(double));
    double* R = calloc((size_t)N * NU * NU, sizeof(double));
    double* M = calloc((size_t)N * NU * NX, sizeof(double));
    double* q = calloc((size_t)N * NX, sizeof(double));
    double* r = calloc((size_t)N * NU, sizeof(double));
    double* K = calloc((size_t)N * NU * NX, sizeof(double));
    double* kk = calloc((size_t)N * NU, sizeof(double));
    double* P = calloc((size_t)N * NX * NX, sizeof(double));
    double* p = calloc((size_t)N * NX, sizeof(double));
    int bad = -1;
    const int st = direction_step(pb, nch, x, u, lam, ye, rho, mu, hessian, delta, A, B, c, Q, R, M, q, r, dx,
                                  du, lh, K, kk, P, p, &bad, out);
    free(nch); free(A); free(B); free(c); free(Q); free(R); free(M); free(q); free(r);
    free(K); free(kk); free(P); free(p);
    return st;
}

/* ------------------------------------------------------------------------
 * AL multiple-shooting iLQR (Sec. IV, Alg. 1).
 * ---------------------------------------------------------------------- */
int orc_bmpc_solve(const orc_problem* pb, const orc_settings* st, int warm, double* x,
                   double* u, double* lam, double* ye, orc_stats* stats, double* hist,
                   int hist_cap)
{
    const int N = pb->N;
    if (N <= 0 || pb->parent[0] != -1) return ORC_ERR_TOPOLOGY;
    for (int i = 1; i < N; ++i)
        if (pb->parent[i] < 0 || pb->parent[i] >= i) return ORC_ERR_TOPOLOGY;
    int* nch = child_counts(pb);
    const size_t nx = NX, nu = NU;
    double* A = calloc((size_t)N * nx * nx, sizeof(double));
    double* B = calloc((size_t)N * nx * nu, sizeof(double));
    double* c = calloc((size_t)N * nx, sizeof(double));
    double* Q = calloc((size_t)N * nx * nx, sizeof(double));
    double* R = calloc((size_t)N * nu * nu, sizeof(double));
    double* M = calloc((size_t)N * nu * nx, sizeof(double));
    double* q = calloc((size_t)N * nx, sizeof(double));
    double* r = calloc((size_t)N * nu, sizeof(double));
    double* dx = calloc((size_t)N * nx, sizeof(double));
    double* du = calloc((size_t)N * nu, sizeof(double));
    double* lh = calloc((size_t)N * nx, sizeof(double));
    double* K = calloc((size_t)N * nu * nx, sizeof(double));
    double* kk = calloc((size_t)N * nu, sizeof(double));
    double* P = calloc((size_t)N * nx * nx, sizeof(double));
    double* p = calloc((size_t)N * nx, sizeof(double));
    double* xt = calloc((size_t)N * nx, sizeof(double));
    double* ut = calloc((size_t)N * nu, sizeof(double));
    double* lt = calloc((size_t)N * nx, sizeof(double));
    int status = ORC_ERR_MAXITER;
    int bad = -1, nhist = 0;

    double rho = st->rho0, mu = st->mu0;
    double omega = st->omega0, eta = st->eta0;
    double r_kkt = INFINITY, viol = INFINITY, phi_last = 0.0;
    int inner_total = 0, outer = 0, ls_fail = 0, ls_fail_run = 0;

    /* initial point: cold = zero inputs and exact rollout (d = 0); bit 16
     * compares the caller's start with the cold one and keeps the better */
    int start_used = (warm & (1 | 4 | 8)) ? 1 : 0;
    if (warm & 16) {
        double* xs = malloc(sizeof(double) * (size_t)N * nx);
        double* us = malloc(sizeof(double) * (size_t)N * nu);
        double* ls = malloc(sizeof(double) * (size_t)N * nx);
        double* ys = malloc(sizeof(double) * (size_t)N * NG);
        memcpy(xs, x, sizeof(double) * (size_t)N * nx);
        memcpy(us, u, sizeof(double) * (size_t)N * nu);
        memcpy(ls, lam, sizeof(double) * (size_t)N * nx);
        memcpy(ys, ye, sizeof(double) * (size_t)N * NG);
        start_point(pb, nch, 0, x, u, lam, ye, rho);
        const double m_cold = start_measure(pb, x, u, lam, ye, rho);
        memcpy(x, xs, sizeof(double) * (size_t)N * nx);
        memcpy(u, us, sizeof(double) * (size_t)N * nu);
        memcpy(lam, ls, sizeof(double) * (size_t)N * nx);
        memcpy(ye, ys, sizeof(double) * (size_t)N * NG);
        free(xs);
        free(us);
        free(ls);
        free(ys);
        start_point(pb, nch, warm & 15, x, u, lam, ye, rho);
        const double m_given = start_measure(pb, x, u, lam, ye, rho);
        if (m_cold < m_given) {
            start_point(pb, nch, 0, x, u, lam, ye, rho);
            start_used = 0;
        }
    } else {
        start_point(pb, nch, warm, x, u, lam, ye, rho);
    }

    for (outer = 0; outer < st->max_outer; ++outer) {
        for (int inner = 0;; ++inner) {
            r_kkt = orc_kkt(pb, x, u, lam, ye, rho);
            if (!isfinite(r_kkt)) {
                status = ORC_ERR_NONFINITE;
                goto done;
            }
            if (r_kkt <= omega || inner >= st->max_inner) break;
            /* total iteration cap (0 = none): stop before a further step */
            if (st->max_iter_total > 0 && inner_total >= st->max_iter_total) {
                status = ORC_ERR_MAXITER;
                goto done;
            }

            /* search direction, merit slope and the adaptive mu */
            double sl[8];
            int lst = direction_step(pb, nch, x, u, lam, ye, rho, mu, st->hessian, st->eig_floor, A, B, c,
                                     Q, R, M, q, r,
                                     dx, du, lh, K, kk, P, p, &bad, sl);
            if (lst != ORC_OK) {
                status = lst;
                goto done;
            }
            mu = sl[5];
            const double dphi0 = sl[6], phi0 = sl[7];

            /* backtracking (Sec. IV-A): each round evaluates n_alpha trial step
             * sizes 2^-k and keeps the largest accepted one; a further round
             * of smaller steps runs only when a round accepts none */
            double alpha_acc = -1.0, phi_acc = phi0;
            const int rounds = st->ls_rounds > 0 ? st->ls_rounds : 1;
            for (int rd = 0; rd < rounds && alpha_acc < 0.0; ++rd) {
                double alpha = ldexp(1.0, -rd * st->n_alpha);
                for (int ka = 0; ka < st->n_alpha; ++ka, alpha *= 0.5) {
                    for (size_t e = 0; e < (size_t)N * nx; ++e) {
                        xt[e] = x[e] + alpha * dx[e];
                        lt[e] = lam[e] + alpha * (lh[e] - lam[e]);
                    }
                    for (size_t e = 0; e < (size_t)N * nu; ++e) ut[e] = u[e] + alpha * du[e];
                    const double phi = merit_impl(pb, nch, xt, ut, lt, ye, rho, mu);
                    if (phi <= phi0 + st->armijo_beta * alpha * dphi0 && alpha > alpha_acc) {
                        alpha_acc = alpha;
                        phi_acc = phi;
                    }
                }
            }
            if (alpha_acc < 0.0) {
                ls_fail++;
                ls_fail_run++;
                if (ls_fail_run >= st->max_ls_fail) {
                    status = ORC_ERR_LINESEARCH;
                    goto done;
                }
                alpha_acc = ldexp(1.0, -(rounds * st->n_alpha - 1));
                phi_acc = NAN;
            } else {
                ls_fail_run = 0;
            }
            for (size_t e = 0; e < (size_t)N * nx; ++e) {
                x[e] += alpha_acc * dx[e];
                lam[e] += alpha_acc * (lh[e] - lam[e]);
            }
            for (size_t e = 0; e < (size_t)N * nu; ++e) u[e] += alpha_acc * du[e];
            phi_last = phi_acc;
            inner_total++;
            if (hist && nhist < hist_cap) {
                double* hrow = hist + 6 * nhist++;
                hrow[0] = outer;
                hrow[1] = r_kkt;
                hrow[2] = alpha_acc;
                hrow[3] = mu;
                hrow[4] = rho;
                hrow[5] = phi_acc;
            }
        }

        /* outer update (BCL) */
        viol = orc_violation(pb, x, u, ye, rho);
        if (viol <= eta) {
            for (int n = 0; n < N; ++n) {
                double g[NG];
                node_terms_impl(pb, n, nch[n] == 0, x + n * NX, u + n * NU, ye + n * NG, rho, g,
                                NULL, NULL, NULL, NULL);
                for (int s = 0; s < NG; ++s)
                    ye[n * NG + s] = g[s] == -INFINITY ? 0.0 : fmax(0.0, ye[n * NG + s] + rho * g[s]);
            }
            if (fmax(r_kkt, viol) < st->eps_tol) {
                status = ORC_OK;
                outer++;
                goto done;
            }
            omega = omega / pow(rho, st->b_omega);
            eta = eta / pow(rho, st->b_eta);
        } else {
            rho = st->tau * rho;
            omega = st->omega0 / pow(rho, st->a_omega);
            eta = st->eta0 / pow(rho, st->a_eta);
        }
        /* Alg. 1 floors omega at eps_tol; eta gets the same floor: the stopping
         * test only asks c < eps_tol, and a smaller eta would raise rho for a
         * violation that already meets it */
        omega = fmax(omega, st->eps_tol);
        eta = fmax(eta, st->eps_tol);
    }

done:
    if (stats) {
        stats->status = status;
        stats->outer_it = outer;
        stats->inner_it = inner_total;
        stats->ls_failures = ls_fail;
        stats->bad_node = bad;
        stats->start = start_used;
        stats->r_kkt = r_kkt;
        stats->viol = viol;
        stats->rho = rho;
        stats->mu = mu;
        stats->merit = phi_last;
    }
    free(nch); free(A); free(B); free(c); free(Q); free(R); free(M); free(q); free(r);
    free(dx); free(du); free(lh); free(K); free(kk); free(P); free(p); free(xt); free(ut);
    free(lt);
    return status;
}

/* ------------------------------------------------------------------------
 * Shifted warm start after one simulated step (receding horizon).
 * The measured state moves to x0' = F(x0, u_0).  Node n of the new problem
 * stands for the old nodes one stage later on the same scenarios, i.e. its
 * children: every value (state, input, costate, PHR multipliers, reference)
 * becomes the pi-weighted mean over the children (the plain mean if their
 * weights sum to zero); a node whose children are leaves repeats its own
 * input.  Leaves keep their costate and multipliers, extrapolate the
 * reference linearly from the parent, and take the state rolled out from
 * the new parent state and input.
 * ---------------------------------------------------------------------- */
void orc_shift(const orc_problem* pb, const double* x, const double* u, const double* lam,
               const double* ye, const double* x0_meas, double* ref_new, double* x0_new, double* xs,
               double* us, double* lams, double* yes)
{
    const int N = pb->N;
    int* nch = child_counts(pb);
    /* the next initial state: measured, else predicted by the model */
    if (x0_meas)
        memcpy(x0_new, x0_meas, sizeof(double) * NX);
    else
        orc_rk4(&pb->model, pb->x0, u, x0_new, NULL, NULL);
    for (int n = 0; n < N; ++n) {
        if (nch[n] == 0) continue;
        double w = 0.0, wu = 0.0;
        int cnt = 0, cnt_ctrl = 0;
        for (int j = n + 1; j < N; ++j)
            if (pb->parent[j] == n) {
                w += pb->weight[j];
                cnt++;
                if (nch[j] > 0) {
                    wu += pb->weight[j];
                    cnt_ctrl++;
                }
            }
        double sx[NX] = {0}, sl[NX] = {0}, sr[4] = {0}, sy[NG] = {0}, su[NU] = {0};
        for (int j = n + 1; j < N; ++j) {
            if (pb->parent[j] != n) continue;
            const double f = w > 0.0 ? pb->weight[j] / w : 1.0 / cnt;
            for (int a = 0; a < NX; ++a) {
                sx[a] += f * x[j * NX + a];
                sl[a] += f * lam[j * NX + a];
            }
            for (int a = 0; a < 4; ++a) sr[a] += f * pb->ref[j * 4 + a];
            for (int a = 0; a < NG; ++a) sy[a] += f * ye[j * NG + a];
            if (nch[j] > 0) {
                const double fu = wu > 0.0 ? pb->weight[j] / wu : 1.0 / cnt_ctrl;
                for (int a = 0; a < NU; ++a) su[a] += fu * u[j * NU + a];
            }
        }
        for (int a = 0; a < NX; ++a) {
            xs[n * NX + a] = sx[a];
            lams[n * NX + a] = sl[a];
        }
        for (int a = 0; a < 4; ++a) ref_new[n * 4 + a] = sr[a];
        for (int a = 0; a < NG; ++a) yes[n * NG + a] = sy[a];
        for (int a = 0; a < NU; ++a) us[n * NU + a] = cnt_ctrl > 0 ? su[a] : u[n * NU + a];
    }
    for (int a = 0; a < NX; ++a) xs[a] = x0_new[a];
    for (int n = 1; n < N; ++n) {
        if (nch[n] != 0) continue;
        const int p = pb->parent[n];
        for (int a = 0; a < 4; ++a) ref_new[n * 4 + a] = 2.0 * pb->ref[n * 4 + a] - pb->ref[p * 4 + a];
        for (int a = 0; a < NX; ++a) lams[n * NX + a] = lam[n * NX + a];
        for (int a = 0; a < NG; ++a) yes[n * NG + a] = ye[n * NG + a];
        for (int a = 0; a < NU; ++a) us[n * NU + a] = 0.0;
    }
    /* leaves: roll out from the shifted parents (parents precede children) */
    for (int n = 1; n < N; ++n)
        if (nch[n] == 0) {
            const int p = pb->parent[n];
            orc_rk4(&pb->model, xs + p * NX, us + p * NU, xs + n * NX, NULL, NULL);
        }
    free(nch);
}
