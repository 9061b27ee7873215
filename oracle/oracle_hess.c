/*
 * Oracle: the pieces of the exact Hessian with eigenvalue modification
 * (Sec. IV-A, search direction: the Hessian of the Lagrangian, made
 * positive definite by modifying its eigenvalues).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 *   - second derivatives of the RK4 bicycle step contracted with a
 *     multiplier, by hyper-dual numbers: a + b e1 + c e2 + d e1 e2 with
 *     e1^2 = e2^2 = 0.  Seeding e1 along z_i and e2 along z_j, the e1 e2 part
 *     of F(z) is d^2 F / dz_i dz_j, exactly up to rounding (no truncation
 *     error, unlike finite differences);
 *   - the symmetric eigendecomposition by the cyclic Jacobi method
 *     (Golub and Van Loan, Sec. 8.5), swept until the off-diagonal part is
 *     negligible;
 *   - the modification itself: eigenvalues below delta are raised to delta.
 */
#include <math.h>
#include <string.h>

#include "oracle.h"

#define NX ORC_NX
#define NU ORC_NU
#define NZ (ORC_NX + ORC_NU)

typedef struct {
    double a, b, c, d;
} hd;

static hd hd_const(double v) { hd r = {v, 0.0, 0.0, 0.0}; return r; }
static hd hd_add(hd x, hd y) { hd r = {x.a + y.a, x.b + y.b, x.c + y.c, x.d + y.d}; return r; }
static hd hd_scale(double s, hd x) { hd r = {s * x.a, s * x.b, s * x.c, s * x.d}; return r; }
static hd hd_mul(hd x, hd y)
{
    hd r = {x.a * y.a, x.a * y.b + x.b * y.a, x.a * y.c + x.c * y.a,
            x.a * y.d + x.b * y.c + x.c * y.b + x.d * y.a};
    return r;
}
/* g(x) for a scalar function with value g0 and derivatives g1, g2 at x.a */
static hd hd_fn(hd x, double g0, double g1, double g2)
{
    hd r = {g0, g1 * x.b, g1 * x.c, g1 * x.d + g2 * x.b * x.c};
    return r;
}
static hd hd_sin(hd x) { return hd_fn(x, sin(x.a), cos(x.a), -sin(x.a)); }
static hd hd_cos(hd x) { return hd_fn(x, cos(x.a), -sin(x.a), -cos(x.a)); }
static hd hd_tan(hd x)
{
    const double t = tan(x.a), s2 = 1.0 + t * t;
    return hd_fn(x, t, s2, 2.0 * t * s2);
}

/* continuous bicycle  [v cos psi, v sin psi, v tan(delta) / L, a] */
static void bicycle_hd(double L, const hd* x, const hd* u, hd* f)
{
    f[0] = hd_mul(x[3], hd_cos(x[2]));
    f[1] = hd_mul(x[3], hd_sin(x[2]));
    f[2] = hd_scale(1.0 / L, hd_mul(x[3], hd_tan(u[1])));
    f[3] = u[0];
}

/* one RK4 step with the input held */
static void rk4_hd(double h, double L, const hd* x, const hd* u, hd* xn)
{
    hd k[4][NX], X[NX];
    static const double stage_c[4] = {0.0, 0.5, 0.5, 1.0};
    for (int st = 0; st < 4; ++st) {
        for (int a = 0; a < NX; ++a)
            X[a] = st ? hd_add(x[a], hd_scale(stage_c[st] * h, k[st - 1][a])) : x[a];
        bicycle_hd(L, X, u, k[st]);
    }
    for (int a = 0; a < NX; ++a) {
        hd s = hd_add(hd_add(k[0][a], hd_scale(2.0, k[1][a])), hd_add(hd_scale(2.0, k[2][a]), k[3][a]));
        xn[a] = hd_add(x[a], hd_scale(h / 6.0, s));
    }
}

void orc_rk4_hessian(const orc_model* m, const double* x, const double* u, const double* mu, double* H)
{
    memset(H, 0, sizeof(double) * NZ * NZ);
    if (m->model == 1) return; /* linear model: no curvature */
    for (int i = 0; i < NZ; ++i)
        for (int j = i; j < NZ; ++j) {
            hd z[NZ], xn[NX];
            for (int k = 0; k < NZ; ++k) {
                z[k] = hd_const(k < NX ? x[k] : u[k - NX]);
                if (k == i) z[k].b = 1.0;
                if (k == j) z[k].c = 1.0;
            }
            rk4_hd(m->dt, m->wheelbase, z, z + NX, xn);
            double s = 0.0;
            for (int a = 0; a < NX; ++a) s += mu[a] * xn[a].d;
            H[i * NZ + j] = s;
            H[j * NZ + i] = s;
        }
}

int orc_sym_eig(int n, const double* A, double* w, double* V)
{
    double S[NZ * NZ];
    if (n <= 0 || n > NZ) return ORC_ERR_INVALID_ARG;
    memcpy(S, A, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += S[i * n + j] * S[i * n + j];
                if (i != j) off += S[i * n + j] * S[i * n + j];
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = S[p * n + q];
                if (apq == 0.0) continue;
                /* rotation that zeroes S[p][q]: t = tan(theta), the smaller
                 * root of t^2 + 2 tau t - 1 = 0 */
                const double tau = (S[q * n + q] - S[p * n + p]) / (2.0 * apq);
                const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) { /* S <- S J (columns p, q) */
                    const double skp = S[k * n + p], skq = S[k * n + q];
                    S[k * n + p] = c * skp - s * skq;
                    S[k * n + q] = s * skp + c * skq;
                }
                for (int k = 0; k < n; ++k) { /* S <- J^T S (rows p, q) */
                    const double spk = S[p * n + k], sqk = S[q * n + k];
                    S[p * n + k] = c * spk - s * sqk;
                    S[q * n + k] = s * spk + c * sqk;
                }
                for (int k = 0; k < n; ++k) { /* V <- V J */
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) w[i] = S[i * n + i];
    return ORC_OK;
}

int orc_eig_modify(int n, const double* A, double delta, double* out)
{
    double w[NZ], V[NZ * NZ];
    const int st = orc_sym_eig(n, A, w, V);
    if (st != ORC_OK) return st;
    for (int i = 0; i < n; ++i) w[i] = w[i] < delta ? delta : w[i];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += V[i * n + k] * w[k] * V[j * n + k];
            out[i * n + j] = s;
        }
    return ORC_OK;
}
