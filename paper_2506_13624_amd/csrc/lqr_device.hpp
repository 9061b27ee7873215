// Device building blocks of the tree Riccati recursion with one node per
// lane and everything in registers.  Used by the tree-LQR kernels and by the
// branch-MPC solver.
#pragma once

#include <hip/hip_runtime.h>

#include "bmpc_internal.hpp"

namespace bmpc {

template <class T = double>
struct LqrArgsT {
    const T* __restrict__ A;
    const T* __restrict__ B;
    const T* __restrict__ c;
    const T* __restrict__ Q;
    const T* __restrict__ R;
    const T* __restrict__ M;
    const T* __restrict__ q;
    const T* __restrict__ r;
    const T* __restrict__ x0;
    T* __restrict__ x;
    T* __restrict__ u;
    T* __restrict__ lam;
    T* __restrict__ K;
    T* __restrict__ k;
    T* __restrict__ P;
    T* __restrict__ p;
    int* bad;      // smallest node whose H was not positive definite (INT_MAX: none)
    int* bad_out;  // copy of *bad taken after the backward pass
};
using LqrArgs = LqrArgsT<double>;

// Cholesky H = L L^T in place (lower triangle used); inv receives the
// reciprocals of the diagonal of L.  False if H is not numerically positive
// definite.
template <int n, class T = double>
__device__ __forceinline__ bool chol_inplace(T (&H)[n][n], T (&inv)[n])
{
    bool ok = true;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        T d = H[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= H[j][k] * H[j][k];
        ok = ok && (d > T(0));
        d = sqrt(d > T(0) ? d : T(1));
        H[j][j] = d;
        inv[j] = T(1) / d;
#pragma unroll
        for (int i = j + 1; i < n; ++i) {
            T s = H[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= H[i][k] * H[j][k];
            H[i][j] = s * inv[j];
        }
    }
    return ok;
}

// The same factorisation with the reciprocal square roots taken from the
// hardware estimate (v_rsq_f64) refined by two Newton steps
// y <- y + y (1 - d y^2) / 2, each of which squares the relative error:
// a shorter dependent chain than a correctly rounded square root followed by
// a division, and within a few units in the last place of it.
__device__ __forceinline__ double rsqrt_refined(double d)
{
    double y = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-d * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

template <int n>
__device__ __forceinline__ bool chol_inplace_rsq(double (&H)[n][n], double (&inv)[n])
{
    bool ok = true;
#pragma unroll
    for (int j = 0; j < n; ++j) {
        double d = H[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= H[j][k] * H[j][k];
        ok = ok && (d > 0.0);
        const double y = rsqrt_refined(d > 0.0 ? d : 1.0);
        inv[j] = y;
        H[j][j] = (d > 0.0 ? d : 1.0) * y;
#pragma unroll
        for (int i = j + 1; i < n; ++i) {
            double s = H[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= H[i][k] * H[j][k];
            H[i][j] = s * y;
        }
    }
    return ok;
}

// The two halves of chol_solve: v <- L^-1 v and v <- L^-T v.
template <int n>
__device__ __forceinline__ void chol_fwd(const double (&L)[n][n], const double (&inv)[n], double (&v)[n])
{
#pragma unroll
    for (int i = 0; i < n; ++i) {
        double s = v[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * v[k];
        v[i] = s * inv[i];
    }
}
template <int n>
__device__ __forceinline__ void chol_bwd(const double (&L)[n][n], const double (&inv)[n], double (&v)[n])
{
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {
        double s = v[i];
#pragma unroll
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * v[k];
        v[i] = s * inv[i];
    }
}

// Solve (L L^T) v = v in place, given the reciprocal diagonal.
template <int n, class T = double>
__device__ __forceinline__ void chol_solve(const T (&L)[n][n], const T (&inv)[n], T (&v)[n])
{
#pragma unroll
    for (int i = 0; i < n; ++i) {
        T s = v[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * v[k];
        v[i] = s * inv[i];
    }
#pragma unroll
    for (int i = n - 1; i >= 0; --i) {
        T s = v[i];
#pragma unroll
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * v[k];
        v[i] = s * inv[i];
    }
}

// Stage cost of one node in registers.
template <int NX, int NU, class T = double>
struct StageRegs {
    T Q[NX][NX], q[NX], R[NU][NU], M[NU][NX], r[NU];
};

// Data of one edge (A, B of the transition, c of the child) in registers.
template <int NX, int NU, class T = double>
struct EdgeRegs {
    T A[NX][NX], B[NX][NU], c[NX];
};

template <int NX, int NU, int LAY, class T>
__device__ __forceinline__ void load_stage(const LqrArgsT<T>& a, int N, int n, StageRegs<NX, NU, T>& s)
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) s.Q[i][j] = a.Q[lidx<LAY>(n, i * NX + j, NX * NX, N)];
        s.q[i] = a.q[lidx<LAY>(n, i, NX, N)];
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) {
#pragma unroll
        for (int j = 0; j < NU; ++j) s.R[i][j] = a.R[lidx<LAY>(n, i * NU + j, NU * NU, N)];
#pragma unroll
        for (int j = 0; j < NX; ++j) s.M[i][j] = a.M[lidx<LAY>(n, i * NX + j, NU * NX, N)];
        s.r[i] = a.r[lidx<LAY>(n, i, NU, N)];
    }
}

// Edge into child j; with SHARED_AB the Jacobians are stored once at the
// parent n (all out-edges of n share the linearisation point) while the
// defect c stays per child.
template <int NX, int NU, int LAY, bool SHARED_AB, class T>
__device__ __forceinline__ void load_edge(const LqrArgsT<T>& a, int N, int n, int j, EdgeRegs<NX, NU, T>& e)
{
    const int ab = SHARED_AB ? n : j;
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int k = 0; k < NX; ++k) e.A[i][k] = a.A[lidx<LAY>(ab, i * NX + k, NX * NX, N)];
#pragma unroll
        for (int k = 0; k < NU; ++k) e.B[i][k] = a.B[lidx<LAY>(ab, i * NU + k, NX * NU, N)];
        e.c[i] = a.c[lidx<LAY>(j, i, NX, N)];
    }
}

template <int NX, int LAY, class T>
__device__ __forceinline__ void load_value(const T* __restrict__ Pg, const T* __restrict__ pg,
                                           int N, int j, T (&P)[NX][NX], T (&p)[NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int k = 0; k < NX; ++k) P[i][k] = Pg[lidx<LAY>(j, i * NX + k, NX * NX, N)];
        p[i] = pg[lidx<LAY>(j, i, NX, N)];
    }
}

template <int NX, int LAY, class T>
__device__ __forceinline__ void store_value(const LqrArgsT<T>& a, int N, int n, const T (&P)[NX][NX],
                                            const T (&p)[NX])
{
#pragma unroll
    for (int i = 0; i < NX; ++i) {
#pragma unroll
        for (int j = 0; j < NX; ++j) a.P[lidx<LAY>(n, i * NX + j, NX * NX, N)] = P[i][j];
        a.p[lidx<LAY>(n, i, NX, N)] = p[i];
    }
}

// Accumulator of one Riccati step: W = Q + sum A^T P A, w, H, G, g.
template <int NX, int NU, class T = double>
struct RicAcc {
    T H[NU][NU], G[NU][NX], g[NU], W[NX][NX], w[NX];

    __device__ __forceinline__ void init(const StageRegs<NX, NU, T>& s)
    {
#pragma unroll
        for (int i = 0; i < NU; ++i) {
#pragma unroll
            for (int j = 0; j < NU; ++j) H[i][j] = s.R[i][j];
#pragma unroll
            for (int j = 0; j < NX; ++j) G[i][j] = s.M[i][j];
            g[i] = s.r[i];
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int j = 0; j < NX; ++j) W[i][j] = s.Q[i][j];
            w[i] = s.q[i];
        }
    }

    // add the child's value function (P, p) seen through edge e
    __device__ __forceinline__ void add_child(const EdgeRegs<NX, NU, T>& e, const T (&P)[NX][NX],
                                              const T (&p)[NX])
    {
        T s[NX], PA[NX][NX], PB[NX][NU];
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            T acc = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) acc += P[i][k] * e.c[k];
            s[i] = p[i] + acc;
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                T t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += P[i][k] * e.A[k][b];
                PA[i][b] = t;
            }
#pragma unroll
            for (int b = 0; b < NU; ++b) {
                T t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += P[i][k] * e.B[k][b];
                PB[i][b] = t;
            }
        }
#pragma unroll
        for (int i = 0; i < NU; ++i) {
#pragma unroll
            for (int b = 0; b < NU; ++b) {
                T t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += e.B[k][i] * PB[k][b];
                H[i][b] += t;
            }
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                T t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += e.B[k][i] * PA[k][b];
                G[i][b] += t;
            }
            T t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) t += e.B[k][i] * s[k];
            g[i] += t;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                T t = 0.0;
#pragma unroll
                for (int k = 0; k < NX; ++k) t += e.A[k][i] * PA[k][b];
                W[i][b] += t;
            }
            T t = 0.0;
#pragma unroll
            for (int k = 0; k < NX; ++k) t += e.A[k][i] * s[k];
            w[i] += t;
        }
    }

    // gains K = -H^-1 G, k = -H^-1 g and the new value function; returns
    // false if H is not positive definite
    __device__ __forceinline__ bool finish(T (&Kn)[NU][NX], T (&kn)[NU], T (&P)[NX][NX],
                                          T (&p)[NX]) const
    {
        T L[NU][NU], inv[NU];
#pragma unroll
        for (int i = 0; i < NU; ++i)
#pragma unroll
            for (int j = 0; j < NU; ++j) L[i][j] = H[i][j];
        const bool ok = chol_inplace<NU>(L, inv);
#pragma unroll
        for (int b = 0; b < NX; ++b) {
            T v[NU];
#pragma unroll
            for (int i = 0; i < NU; ++i) v[i] = G[i][b];
            chol_solve<NU>(L, inv, v);
#pragma unroll
            for (int i = 0; i < NU; ++i) Kn[i][b] = -v[i];
        }
        {
            T v[NU];
#pragma unroll
            for (int i = 0; i < NU; ++i) v[i] = g[i];
            chol_solve<NU>(L, inv, v);
#pragma unroll
            for (int i = 0; i < NU; ++i) kn[i] = -v[i];
        }
        // X = W + G^T K ; P = (X + X^T)/2 ; p = w + G^T k
#pragma unroll
        for (int i = 0; i < NX; ++i) {
#pragma unroll
            for (int b = 0; b < NX; ++b) {
                T t = W[i][b];
#pragma unroll
                for (int rr = 0; rr < NU; ++rr) t += G[rr][i] * Kn[rr][b];
                P[i][b] = t;
            }
            T t = w[i];
#pragma unroll
            for (int rr = 0; rr < NU; ++rr) t += G[rr][i] * kn[rr];
            p[i] = t;
        }
#pragma unroll
        for (int i = 0; i < NX; ++i)
#pragma unroll
            for (int b = i + 1; b < NX; ++b) {
                const T m = 0.5 * (P[i][b] + P[b][i]);
                P[i][b] = m;
                P[b][i] = m;
            }
        return ok;
    }
};

}  // namespace bmpc
