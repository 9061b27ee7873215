// Conditional value functions (Sec. II-A, eqs. V_ki_min / sol_min): the
// tuple (A, c, C, P, p) of
//   V_{k->i}(x_k, x_i) = max_lam 1/2 x_k^T P x_k + p^T x_k - 1/2 lam^T C lam + lam^T (x_i - A x_k - c)
// and their associative composition, in registers (one element per lane).
//
// The composition is the minimisation over the intermediate state (eq.
// V_ki_min); with E = I + C_kj P_ji it reads
//   A = A_ji E^-1 A_kj,  c = A_ji E^-1 (c_kj - C_kj p_ji) + c_ji,  C = A_ji E^-1 C_kj A_ji^T + C_ji,
//   P = A_kj^T P_ji E^-1 A_kj + P_kj,  p = A_kj^T E^-T (p_ji + P_ji c_kj) + p_kj,
// (the printed signs of eq. comb_rule are corrected; P_ji E^-1 = E^-T P_ji by
// symmetry of C and P, so one LU of E serves every term).
#pragma once

#include <hip/hip_runtime.h>

#include "lqr_device.hpp"  // chol_inplace, chol_solve

namespace bmpc {

template <int NX>
struct Cvf {
    double A[NX][NX], c[NX], C[NX][NX], P[NX][NX], p[NX];
};

// LU with partial pivoting of an NX x NX matrix, in place; piv records the
// row order.  Returns false for a (numerically) singular matrix.
template <int n>
__device__ __forceinline__ bool lu_pp(double (&E)[n][n], int (&piv)[n])
{
    bool ok = true;
#pragma unroll
    for (int i = 0; i < n; ++i) piv[i] = i;
#pragma unroll
    for (int k = 0; k < n; ++k) {
        int best = k;
        double bv = fabs(E[k][k]);
#pragma unroll
        for (int i = k + 1; i < n; ++i)
            if (fabs(E[i][k]) > bv) {
                bv = fabs(E[i][k]);
                best = i;
            }
        if (best != k) {
#pragma unroll
            for (int j = 0; j < n; ++j) {
                const double t = E[k][j];
                E[k][j] = E[best][j];
                E[best][j] = t;
            }
            const int t = piv[k];
            piv[k] = piv[best];
            piv[best] = t;
        }
        ok = ok && (bv > 0.0);
        const double inv = 1.0 / (bv > 0.0 ? E[k][k] : 1.0);
#pragma unroll
        for (int i = k + 1; i < n; ++i) {
            const double f = E[i][k] * inv;
            E[i][k] = f;
#pragma unroll
            for (int j = k + 1; j < n; ++j) E[i][j] -= f * E[k][j];
        }
    }
    return ok;
}

// x = E^-1 b with the factors of lu_pp
template <int n>
__device__ __forceinline__ void lu_solve(const double (&LU)[n][n], const int (&piv)[n], const double (&b)[n],
                                         double (&x)[n])
{
    double y[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        double s = b[piv[i]];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= LU[i][k] * y[k];
        y[i] = s;
    }
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < n; ++k) s -= LU[i][k] * x[k];
        x[i] = s / LU[i][i];
    }
}

// x = E^-T b with the factors of lu_pp (E = P^T L U, so E^T = U^T L^T P)
template <int n>
__device__ __forceinline__ void lu_solve_t(const double (&LU)[n][n], const int (&piv)[n], const double (&b)[n],
                                           double (&x)[n])
{
    double z[n], w[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {  // U^T z = b
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= LU[k][i] * z[k];
        z[i] = s / LU[i][i];
    }
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {  // L^T w = z (unit diagonal)
        double s = z[i];
#pragma unroll
        for (int k = i + 1; k < n; ++k) s -= LU[k][i] * w[k];
        w[i] = s;
    }
#pragma unroll
    for (int i = 0; i < n; ++i) x[piv[i]] = w[i];
}

// One-step element of a node with stage cost (Q, R, M, q, r) and the edge
// x' = A x + B u + c to its only child (minimisation over u; needs R > 0).
// Returns false if R is not positive definite.
template <int NX, int NU>
__device__ __forceinline__ bool cvf_element(const double (&Q)[NX][NX], const double (&R)[NU][NU],
                                            const double (&M)[NU][NX], const double (&q)[NX],
                                            const double (&r)[NU], const double (&A)[NX][NX],
                                            const double (&B)[NX][NU], const double (&c)[NX], Cvf<NX>& e)
{
    double L[NU][NU], inv[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i)
#pragma unroll
        for (int j = 0; j < NU; ++j) L[i][j] = R[i][j];
    const bool ok = chol_inplace<NU>(L, inv);
    // Ri_M = R^-1 M (NU x NX), Ri_r = R^-1 r, Ri_Bt = R^-1 B^T (NU x NX)
    double RiM[NU][NX], RiBt[NU][NX], Rir[NU];
#pragma unroll
    for (int b = 0; b < NX; ++b) {
        double v[NU], w[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            v[i] = M[i][b];
            w[i] = B[b][i];
        }
        chol_solve<NU>(L, inv, v);
        chol_solve<NU>(L, inv, w);
#pragma unroll
        for (int i = 0; i < NU; ++i) {
            RiM[i][b] = v[i];
            RiBt[i][b] = w[i];
        }
    }
    {
        double v[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i) v[i] = r[i];
        chol_solve<NU>(L, inv, v);
#pragma unroll
        for (int i = 0; i < NU; ++i) Rir[i] = v[i];
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        double ci = c[i];
#pragma unroll
        for (int k = 0; k < NU; ++k) ci -= B[i][k] * Rir[k];
        e.c[i] = ci;
        double pi = q[i];
#pragma unroll
        for (int k = 0; k < NU; ++k) pi -= M[k][i] * Rir[k];
        e.p[i] = pi;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double a = A[i][j], cc = 0.0, pp = Q[i][j];
#pragma unroll
            for (int k = 0; k < NU; ++k) {
                a -= B[i][k] * RiM[k][j];
                cc += B[i][k] * RiBt[k][j];
                pp -= M[k][i] * RiM[k][j];
            }
            e.A[i][j] = a;
            e.C[i][j] = cc;
            e.P[i][j] = pp;
        }
    }
    return ok;
}

// out = a (+) b
template <int NX>
__device__ __forceinline__ void cvf_combine(const Cvf<NX>& a, const Cvf<NX>& b, Cvf<NX>& out)
{
    double E[NX][NX];
    int piv[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) s += a.C[i][k] * b.P[k][j];
            E[i][j] = s;
        }
    lu_pp<NX>(E, piv);
    // X = E^-1 A_a, Y = E^-1 C_a (column by column), y = E^-1 (c_a - C_a p_b)
    double X[NX][NX], Y[NX][NX], y[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
        double col[NX], sol[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) col[i] = a.A[i][j];
        lu_solve<NX>(E, piv, col, sol);
#pragma unroll
        for (int i = 0; i < NX; ++i) X[i][j] = sol[i];
#pragma unroll
        for (int i = 0; i < NX; ++i) col[i] = a.C[i][j];
        lu_solve<NX>(E, piv, col, sol);
#pragma unroll
        for (int i = 0; i < NX; ++i) Y[i][j] = sol[i];
    }
    {
        double v[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double s = a.c[i];
#pragma unroll
            for (int k = 0; k < NX; ++k) s -= a.C[i][k] * b.p[k];
            v[i] = s;
        }
        lu_solve<NX>(E, piv, v, y);
    }
    // z = E^-T (p_b + P_b c_a)
    double z[NX];
    {
        double v[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double s = b.p[i];
#pragma unroll
            for (int k = 0; k < NX; ++k) s += b.P[i][k] * a.c[k];
            v[i] = s;
        }
        lu_solve_t<NX>(E, piv, v, z);
    }
    // P_b X (for P) and A_b Y (for C)
    double PX[NX][NX], AY[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double s = 0.0, t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                s += b.P[i][k] * X[k][j];
                t += b.A[i][k] * Y[k][j];
            }
            PX[i][j] = s;
            AY[i][j] = t;
        }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        double cs = b.c[i], ps = a.p[i];
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            cs += b.A[i][k] * y[k];
            ps += a.A[k][i] * z[k];
        }
        out.c[i] = cs;
        out.p[i] = ps;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double av = 0.0, cv = b.C[i][j], pv = a.P[i][j];
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                av += b.A[i][k] * X[k][j];
                cv += AY[i][k] * b.A[j][k];
                pv += a.A[k][i] * PX[k][j];
            }
            out.A[i][j] = av;
            out.C[i][j] = cv;
            out.P[i][j] = pv;
        }
    }
    // keep the symmetric parts exactly symmetric
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = i + 1; j < NX; ++j) {
            const double cm = 0.5 * (out.C[i][j] + out.C[j][i]);
            const double pm = 0.5 * (out.P[i][j] + out.P[j][i]);
            out.C[i][j] = out.C[j][i] = cm;
            out.P[i][j] = out.P[j][i] = pm;
        }
}

// Value function V_k = a (+) (0, 0, 0, Pv, pv): only P and p of the result.
template <int NX>
__device__ __forceinline__ void cvf_apply_value(const Cvf<NX>& a, const double (&Pv)[NX][NX], const double (&pv)[NX],
                                                double (&P)[NX][NX], double (&p)[NX])
{
    double E[NX][NX];
    int piv[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double s = (i == j) ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) s += a.C[i][k] * Pv[k][j];
            E[i][j] = s;
        }
    lu_pp<NX>(E, piv);
    double X[NX][NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) {
        double col[NX], sol[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) col[i] = a.A[i][j];
        lu_solve<NX>(E, piv, col, sol);
#pragma unroll
        for (int i = 0; i < NX; ++i) X[i][j] = sol[i];
    }
    double z[NX];
    {
        double v[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double s = pv[i];
#pragma unroll
            for (int k = 0; k < NX; ++k) s += Pv[i][k] * a.c[k];
            v[i] = s;
        }
        lu_solve_t<NX>(E, piv, v, z);
    }
    double PX[NX][NX];
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double s = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) s += Pv[i][k] * X[k][j];
            PX[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
        double ps = a.p[i];
#pragma unroll
        for (int k = 0; k < NX; ++k) ps += a.A[k][i] * z[k];
        p[i] = ps;
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            double pv2 = a.P[i][j];
#pragma unroll
            for (int k = 0; k < NX; ++k) pv2 += a.A[k][i] * PX[k][j];
            P[i][j] = pv2;
        }
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int j = i + 1; j < NX; ++j) {
            const double m = 0.5 * (P[i][j] + P[j][i]);
            P[i][j] = P[j][i] = m;
        }
}

}  // namespace bmpc
