// Device building blocks of the tree Riccati recursion (one node per lane,
// everything in registers).  Used by the tree-LQR kernels and by the
// branch-MPC solver.
#pragma once

#include <hip/hip_runtime.h>

#include "bmpc_internal.hpp"

namespace bmpc {

struct LqrArgs {
    const double *A, *B, *c, *Q, *R, *M, *q, *r, *x0;
    double *x, *u, *lam, *K, *k, *P, *p;
    int* bad;
};

// Cholesky H = L L^T in place (lower triangle used).  False if H is not
// numerically positive definite.
template <int n>
__device__ __forceinline__ bool chol_inplace(double (&H)[n][n])
{
    bool ok = true;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        double d = H[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= H[j][k] * H[j][k];
        ok = ok && (d > 0.0);
        d = sqrt(d > 0.0 ? d : 1.0);
        H[j][j] = d;
        const double inv = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < n; ++i) {
            double s = H[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= H[i][k] * H[j][k];
            H[i][j] = s * inv;
        }
    }
    return ok;
}

// Solve (L L^T) v = v in place.
template <int n>
__device__ __forceinline__ void chol_solve(const double (&L)[n][n], double (&v)[n])
{
#pragma unroll
    for (int i = 0; i < n; ++i) {
        double s = v[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * v[k];
        v[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {
        double s = v[i];
#pragma unroll
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * v[k];
        v[i] = s / L[i][i];
    }
}

template <int NX, int NU, int LAY>
__device__ __forceinline__ void leaf_value(const LqrArgs& a, int N, int n, double (&P)[NX][NX],
                                           double (&p)[NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) P[i][j] = a.Q[lidx<LAY>(n, i * NX + j, NX * NX, N)];
        p[i] = a.q[lidx<LAY>(n, i, NX, N)];
    }
#pragma unroll
    for (int e = 0; e < NU * NX; ++e) a.K[lidx<LAY>(n, e, NU * NX, N)] = 0.0;
#pragma unroll
    for (int e = 0; e < NU; ++e) a.k[lidx<LAY>(n, e, NU, N)] = 0.0;
}

template <int NX, int LAY>
__device__ __forceinline__ void store_value(const LqrArgs& a, int N, int n, const double (&P)[NX][NX],
                                            const double (&p)[NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) a.P[lidx<LAY>(n, i * NX + j, NX * NX, N)] = P[i][j];
        a.p[lidx<LAY>(n, i, NX, N)] = p[i];
    }
}

// Riccati step at control node n with children c0..c1-1.  If use_regs, the
// single child's value function is already in (P, p); otherwise every
// child's is read from a.P / a.p in child order.  With SHARED_AB the
// Jacobians (A, B) of all out-edges of n are stored once at n (siblings
// share the linearisation point) and c stays per child.
template <int NX, int NU, int LAY, bool SHARED_AB>
__device__ __forceinline__ void riccati_node(const LqrArgs& a, int N, int n, int c0, int c1,
                                             bool use_regs, double (&P)[NX][NX], double (&p)[NX])
{
    double H[NU][NU], G[NU][NX], g[NU], W[NX][NX], w[NX];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
#pragma unroll
        for (int j = 0; j < NU; ++j) H[i][j] = a.R[lidx<LAY>(n, i * NU + j, NU * NU, N)];
#pragma unroll
        for (int j = 0; j < NX; ++j) G[i][j] = a.M[lidx<LAY>(n, i * NX + j, NU * NX, N)];
        g[i] = a.r[lidx<LAY>(n, i, NU, N)];
    }
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) W[i][j] = a.Q[lidx<LAY>(n, i * NX + j, NX * NX, N)];
        w[i] = a.q[lidx<LAY>(n, i, NX, N)];
    }
    for (int j = c0; j < c1; ++j) {
        if (!use_regs) {
#pragma unroll
            for (int i = 0; i < NX; ++i) {
#pragma unroll
                for (int k = 0; k < NX; ++k) P[i][k] = a.P[lidx<LAY>(j, i * NX + k, NX * NX, N)];
                p[i] = a.p[lidx<LAY>(j, i, NX, N)];
            }
        }
        const int e = SHARED_AB ? n : j;
        double Am[NX][NX], Bm[NX][NU], cv[NX];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int k = 0; k < NX; ++k) Am[i][k] = a.A[lidx<LAY>(e, i * NX + k, NX * NX, N)];
#pragma unroll
            for (int k = 0; k < NU; ++k) Bm[i][k] = a.B[lidx<LAY>(e, i * NU + k, NX * NU, N)];
            cv[i] = a.c[lidx<LAY>(j, i, NX, N)];
        }
        // s = p + P c ; PA = P A ; PB = P B
        double s[NX], PA[NX][NX], PB[NX][NU];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) acc += P[i][k] * cv[k];
            s[i] = p[i] + acc;
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += P[i][k] * Am[k][b];
                PA[i][b] = t;
            }
#pragma unroll
            for (int b = 0; b < NU; ++b) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += P[i][k] * Bm[k][b];
                PB[i][b] = t;
            }
        }
#pragma unroll
        for (int i = 0; i < NU; ++i) {
#pragma unroll
            for (int b = 0; b < NU; ++b) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += Bm[k][i] * PB[k][b];
                H[i][b] += t;
            }
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += Bm[k][i] * PA[k][b];
                G[i][b] += t;
            }
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) t += Bm[k][i] * s[k];
            g[i] += t;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += Am[k][i] * PA[k][b];
                W[i][b] += t;
            }
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) t += Am[k][i] * s[k];
            w[i] += t;
        }
    }
    double L[NU][NU];
#pragma unroll
    for (int i = 0; i < NU; ++i)
#pragma unroll
        for (int j = 0; j < NU; ++j) L[i][j] = H[i][j];
    if (!chol_inplace<NU>(L)) atomicMin(a.bad, n);
    double Kn[NU][NX], kn[NU];
#pragma unroll
    for (int b = 0; b < NX; ++b) {
        double v[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i) v[i] = G[i][b];
        chol_solve<NU>(L, v);
#pragma unroll
        for (int i = 0; i < NU; ++i) Kn[i][b] = -v[i];
    }
    {
        double v[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i) v[i] = g[i];
        chol_solve<NU>(L, v);
#pragma unroll
        for (int i = 0; i < NU; ++i) kn[i] = -v[i];
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) {
#pragma unroll
        for (int b = 0; b < NX; ++b) a.K[lidx<LAY>(n, i * NX + b, NU * NX, N)] = Kn[i][b];
        a.k[lidx<LAY>(n, i, NU, N)] = kn[i];
    }
    // X = W + G^T K ; P = (X + X^T)/2 ; p = w + G^T k
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int b = 0; b < NX; ++b) {
            double t = W[i][b];
#pragma unroll
            for (int r = 0; r < NU; ++r) t += G[r][i] * Kn[r][b];
            P[i][b] = t;
        }
        double t = w[i];
#pragma unroll
        for (int r = 0; r < NU; ++r) t += G[r][i] * kn[r];
        p[i] = t;
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int b = i + 1; b < NX; ++b) {
            const double m = 0.5 * (P[i][b] + P[b][i]);
            P[i][b] = m;
            P[b][i] = m;
        }
}

}  // namespace bmpc
