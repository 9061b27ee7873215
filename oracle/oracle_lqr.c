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

/* the recursion in double ... */
#define REAL double
#define SQRT sqrt
#define CHOL chol_d
#define CHOL_SOLVE chol_solve_d
#define LQR tree_lqr_d
#include "oracle_lqr_impl.h"
#undef REAL
#undef SQRT
#undef CHOL
#undef CHOL_SOLVE
#undef LQR

/* ... and in long double (x87 extended precision, 64-bit significand), for
 * reference solutions of badly conditioned problems: the distance between
 * the double recursion and this one measures the rounding floor of double
 * arithmetic on a given problem */
#define REAL long double
#define SQRT sqrtl
#define CHOL chol_ld
#define CHOL_SOLVE chol_solve_ld
#define LQR tree_lqr_ld
#include "oracle_lqr_impl.h"
#undef REAL
#undef SQRT
#undef CHOL
#undef CHOL_SOLVE
#undef LQR

/* and in single precision: the FP32 variant of the recursion, every
 * operation rounded to float in the serial order above */
#define REAL float
#define SQRT sqrtf
#define CHOL chol_f
#define CHOL_SOLVE chol_solve_f
#define LQR tree_lqr_f
#include "oracle_lqr_impl.h"
#undef REAL
#undef SQRT
#undef CHOL
#undef CHOL_SOLVE
#undef LQR

int orc_tree_lqr(int N, int nx, int nu, const int* parent,
                 const double* A, const double* B, const double* c,
                 const double* Q, const double* R, const double* M,
                 const double* q, const double* r, const double* x0,
                 double* x, double* u, double* lam,
                 double* K, double* k, double* P, double* p, int* bad_node)
{
    return tree_lqr_d(N, nx, nu, parent, A, B, c, Q, R, M, q, r, x0, x, u, lam, K, k, P, p, bad_node);
}

/* The recursion in another precision: inputs rounded from double, outputs
 * converted back to double. */
#define ORC_LQR_IN_TYPE(NAME, TYPE, IMPL)                                                            \
    static TYPE* NAME##_widen(const double* a, size_t n)                                             \
    {                                                                                                \
        TYPE* w = malloc(sizeof(TYPE) * (n ? n : 1));                                                \
        for (size_t i = 0; i < n; ++i) w[i] = (TYPE)a[i];                                            \
        return w;                                                                                    \
    }                                                                                                \
    static void NAME##_narrow(const TYPE* a, double* out, size_t n)                                  \
    {                                                                                                \
        for (size_t i = 0; i < n; ++i) out[i] = (double)a[i];                                        \
    }                                                                                                \
    int NAME(int N, int nx, int nu, const int* parent, const double* A, const double* B,            \
             const double* c, const double* Q, const double* R, const double* M, const double* q,   \
             const double* r, const double* x0, double* x, double* u, double* lam, double* K,       \
             double* k, double* P, double* p, int* bad_node)                                         \
    {                                                                                                \
        if (N <= 0 || nx <= 0 || nu <= 0) return ORC_ERR_INVALID_ARG;                               \
        const size_t n = (size_t)N, nn = n * nx * nx, nm = n * nx * nu, mm = n * nu * nu;            \
        TYPE *wA = NAME##_widen(A, nn), *wB = NAME##_widen(B, nm), *wc = NAME##_widen(c, n * nx),   \
             *wQ = NAME##_widen(Q, nn), *wR = NAME##_widen(R, mm), *wM = NAME##_widen(M, nm),        \
             *wq = NAME##_widen(q, n * nx), *wr = NAME##_widen(r, n * nu),                           \
             *wx0 = NAME##_widen(x0, (size_t)nx);                                                    \
        TYPE *ox = malloc(sizeof(TYPE) * n * nx), *ou = malloc(sizeof(TYPE) * n * nu),              \
             *ol = malloc(sizeof(TYPE) * n * nx), *oK = malloc(sizeof(TYPE) * nm),                   \
             *ok = malloc(sizeof(TYPE) * n * nu), *oP = malloc(sizeof(TYPE) * nn),                   \
             *op = malloc(sizeof(TYPE) * n * nx);                                                    \
        const int st = IMPL(N, nx, nu, parent, wA, wB, wc, wQ, wR, wM, wq, wr, wx0, ox, ou, ol, oK, \
                            ok, oP, op, bad_node);                                                   \
        if (st == ORC_OK) {                                                                          \
            NAME##_narrow(ox, x, n * nx);                                                            \
            NAME##_narrow(ou, u, n * nu);                                                            \
            NAME##_narrow(ol, lam, n * nx);                                                          \
            NAME##_narrow(oK, K, nm);                                                                \
            NAME##_narrow(ok, k, n * nu);                                                            \
            NAME##_narrow(oP, P, nn);                                                                \
            NAME##_narrow(op, p, n * nx);                                                            \
        }                                                                                            \
        free(wA); free(wB); free(wc); free(wQ); free(wR); free(wM); free(wq); free(wr); free(wx0);  \
        free(ox); free(ou); free(ol); free(oK); free(ok); free(oP); free(op);                        \
        return st;                                                                                   \
    }

ORC_LQR_IN_TYPE(orc_tree_lqr_ld, long double, tree_lqr_ld)
ORC_LQR_IN_TYPE(orc_tree_lqr_f, float, tree_lqr_f)
