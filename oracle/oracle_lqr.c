/*
 * Oracle: serial tree Riccati recursion for the tree LQR problem.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Problem (tree LQR, Sec. III, eq. lqr_tree_approx, with the stage cost of
 * eq. LQR):  minimise over the state tree x and input tree u
 *   sum_{n control} 1/2 [x;u]^T [[Q, M^T],[M, R]] [x;u] + q^T x + r^T u
 *   + sum_{l leaf} 1/2 x^T Q x + q^T x
 * subject to x_0 = x0 and x_j = A_j x_p + B_j u_p + c_j for every j != 0
 * with p = parent(j).  The dynamics are stored on the child (edge j), which
 * lets siblings carry different dynamics and defects.
 *
 * Method (Sec. III-A, eq. tree_Riccati; gains of eq. tree_feedback_laws):
 * visit nodes leaves-first; the value function of node n is obtained by
 * minimising its stage cost plus the sum of its children's value functions
 * over u_n.  With V_j(x) = 1/2 x^T P_j x + p_j^T x + const:
 *   H = R_n + sum_j B_j^T P_j B_j
 *   G = M_n + sum_j B_j^T P_j A_j
 *   g = r_n + sum_j B_j^T (p_j + P_j c_j)
 *   K_n = -H^{-1} G,   k_n = -H^{-1} g
 *   P_n = Q_n + sum_j A_j^T P_j A_j + G^T K_n      (then symmetrised)
 *   p_n = q_n + sum_j A_j^T (p_j + P_j c_j) + G^T k_n
 * Leaves: P = Q, p = q.  Forward: u_n = K_n x_n + k_n, x_j from the
 * dynamics, and the costate lam_j = P_j x_j + p_j, which is the multiplier of
 * x_j = f_p(.) - ... in the convention  L = cost + lam^T (f - x).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Cholesky H = L L^T in place (lower triangle).  Returns 0 on failure. */
static int chol(int n, double* H)
{
    for (int j = 0; j < n; ++j) {
        double d = H[j * n + j];
        for (int k = 0; k < j; ++k) d -= H[j * n + k] * H[j * n + k];
        if (!(d > 0.0) || !isfinite(d)) return 0;
        d = sqrt(d);
        H[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = H[i * n + j];
            for (int k = 0; k < j; ++k) s -= H[i * n + k] * H[j * n + k];
            H[i * n + j] = s / d;
        }
    }
    return 1;
}

/* Solve (L L^T) z = y in place for one right-hand side. */
static void chol_solve(int n, const double* L, double* y)
{
    for (int i = 0; i < n; ++i) {
        double s = y[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * y[k];
        y[i] = s / L[i * n + i];
    }
}

int orc_tree_lqr(int N, int nx, int nu, const int* parent,
                 const double* A, const double* B, const double* c,
                 const double* Q, const double* R, const double* M,
                 const double* q, const double* r, const double* x0,
                 double* x, double* u, double* lam,
                 double* K, double* k, double* P, double* p, int* bad_node)
{
    if (N <= 0 || nx <= 0 || nu <= 0 || !parent) return ORC_ERR_INVALID_ARG;
    if (parent[0] != -1) return ORC_ERR_TOPOLOGY;
    for (int i = 1; i < N; ++i)
        if (parent[i] < 0 || parent[i] >= i) return ORC_ERR_TOPOLOGY;

    const int nn = nx * nx, nm = nx * nu, mm = nu * nu;
    /* children lists (CSR) in increasing node order */
    int* cnt = calloc((size_t)N + 1, sizeof(int));
    int* kids = malloc(sizeof(int) * (size_t)(N > 1 ? N - 1 : 1));
    int* fill = calloc((size_t)N, sizeof(int));
    double* H = malloc(sizeof(double) * mm);
    double* G = malloc(sizeof(double) * nm);
    double* g = malloc(sizeof(double) * nu);
    double* W = malloc(sizeof(double) * nn);
    double* w = malloc(sizeof(double) * nx);
    double* s = malloc(sizeof(double) * nx);
    double* PA = malloc(sizeof(double) * nn);
    double* PB = malloc(sizeof(double) * nm);
    double* col = malloc(sizeof(double) * nu);
    int status = ORC_OK;

    for (int i = 1; i < N; ++i) cnt[parent[i] + 1]++;
    for (int i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    for (int i = 1; i < N; ++i) kids[cnt[parent[i]] + fill[parent[i]]++] = i;

    /* backward: every child has a larger index than its parent */
    for (int n = N - 1; n >= 0 && status == ORC_OK; --n) {
        double* Pn = P + (size_t)n * nn;
        double* pn = p + (size_t)n * nx;
        double* Kn = K + (size_t)n * nm;
        double* kn = k + (size_t)n * nu;
        if (cnt[n + 1] == cnt[n]) {             /* leaf */
            memcpy(Pn, Q + (size_t)n * nn, sizeof(double) * nn);
            memcpy(pn, q + (size_t)n * nx, sizeof(double) * nx);
            memset(Kn, 0, sizeof(double) * nm);
            memset(kn, 0, sizeof(double) * nu);
            continue;
        }
        memcpy(H, R + (size_t)n * mm, sizeof(double) * mm);
        memcpy(G, M + (size_t)n * nm, sizeof(double) * nm);
        memcpy(g, r + (size_t)n * nu, sizeof(double) * nu);
        memcpy(W, Q + (size_t)n * nn, sizeof(double) * nn);
        memcpy(w, q + (size_t)n * nx, sizeof(double) * nx);
        for (int e = cnt[n]; e < cnt[n + 1]; ++e) {
            const int j = kids[e];
            const double* Pj = P + (size_t)j * nn;
            const double* pj = p + (size_t)j * nx;
            const double* Aj = A + (size_t)j * nn;
            const double* Bj = B + (size_t)j * nm;
            const double* cj = c + (size_t)j * nx;
            for (int a = 0; a < nx; ++a) {
                double acc = pj[a];
                for (int b = 0; b < nx; ++b) acc += Pj[a * nx + b] * cj[b];
                s[a] = acc;
                for (int b = 0; b < nx; ++b) {
                    double t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Pj[a * nx + l] * Aj[l * nx + b];
                    PA[a * nx + b] = t;
                }
                for (int b = 0; b < nu; ++b) {
                    double t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Pj[a * nx + l] * Bj[l * nu + b];
                    PB[a * nu + b] = t;
                }
            }
            for (int a = 0; a < nu; ++a) {
                for (int b = 0; b < nu; ++b) {
                    double t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Bj[l * nu + a] * PB[l * nu + b];
                    H[a * nu + b] += t;
                }
                for (int b = 0; b < nx; ++b) {
                    double t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Bj[l * nu + a] * PA[l * nx + b];
                    G[a * nx + b] += t;
                }
                double t = 0.0;
                for (int l = 0; l < nx; ++l) t += Bj[l * nu + a] * s[l];
                g[a] += t;
            }
            for (int a = 0; a < nx; ++a) {
                for (int b = 0; b < nx; ++b) {
                    double t = 0.0;
                    for (int l = 0; l < nx; ++l) t += Aj[l * nx + a] * PA[l * nx + b];
                    W[a * nx + b] += t;
                }
                double t = 0.0;
                for (int l = 0; l < nx; ++l) t += Aj[l * nx + a] * s[l];
                w[a] += t;
            }
        }
        if (!chol(nu, H)) {
            status = ORC_ERR_NOT_PD;
            if (bad_node) *bad_node = n;
            break;
        }
        /* K = -H^{-1} G column by column, k = -H^{-1} g */
        for (int b = 0; b < nx; ++b) {
            for (int a = 0; a < nu; ++a) col[a] = G[a * nx + b];
            chol_solve(nu, H, col);
            for (int a = 0; a < nu; ++a) Kn[a * nx + b] = -col[a];
        }
        for (int a = 0; a < nu; ++a) col[a] = g[a];
        chol_solve(nu, H, col);
        for (int a = 0; a < nu; ++a) kn[a] = -col[a];
        for (int a = 0; a < nx; ++a) {
            for (int b = 0; b < nx; ++b) {
                double t = W[a * nx + b];
                for (int l = 0; l < nu; ++l) t += G[l * nx + a] * Kn[l * nx + b];
                Pn[a * nx + b] = t;
            }
            double t = w[a];
            for (int l = 0; l < nu; ++l) t += G[l * nx + a] * kn[l];
            pn[a] = t;
        }
        for (int a = 0; a < nx; ++a)
            for (int b = a + 1; b < nx; ++b) {
                double m = 0.5 * (Pn[a * nx + b] + Pn[b * nx + a]);
                Pn[a * nx + b] = m;
                Pn[b * nx + a] = m;
            }
    }

    if (status == ORC_OK) {
        /* forward rollout in increasing node order */
        memcpy(x, x0, sizeof(double) * nx);
        for (int n = 0; n < N; ++n) {
            const double* xn = x + (size_t)n * nx;
            double* un = u + (size_t)n * nu;
            const double* Pn = P + (size_t)n * nn;
            const double* pn = p + (size_t)n * nx;
            double* ln = lam + (size_t)n * nx;
            for (int a = 0; a < nx; ++a) {
                double t = pn[a];
                for (int b = 0; b < nx; ++b) t += Pn[a * nx + b] * xn[b];
                ln[a] = t;
            }
            if (cnt[n + 1] == cnt[n]) {
                memset(un, 0, sizeof(double) * nu);
                continue;
            }
            const double* Kn = K + (size_t)n * nm;
            const double* kn = k + (size_t)n * nu;
            for (int a = 0; a < nu; ++a) {
                double t = kn[a];
                for (int b = 0; b < nx; ++b) t += Kn[a * nx + b] * xn[b];
                un[a] = t;
            }
            for (int e = cnt[n]; e < cnt[n + 1]; ++e) {
                const int j = kids[e];
                const double* Aj = A + (size_t)j * nn;
                const double* Bj = B + (size_t)j * nm;
                const double* cj = c + (size_t)j * nx;
                double* xj = x + (size_t)j * nx;
                for (int a = 0; a < nx; ++a) {
                    double t = cj[a];
                    for (int b = 0; b < nx; ++b) t += Aj[a * nx + b] * xn[b];
                    for (int b = 0; b < nu; ++b) t += Bj[a * nu + b] * un[b];
                    xj[a] = t;
                }
            }
        }
    }

    free(cnt); free(kids); free(fill); free(H); free(G); free(g); free(W); free(w);
    free(s); free(PA); free(PB); free(col);
    return status;
}
